// Serving loop: continuous batching of decode requests (lpdec_server_* in lpdec.h).
//
// One dispatcher thread owns the device side.  Each pass it
//   1. collects completions: scans the per-frame completion flags the kernels write
//      to host-visible memory, finishes requests whose frames are all done, frees
//      their memory and records latency;
//   2. admits queued requests in arrival order (no overtaking, so no starvation)
//      while their footprint fits the budget: each frame reserves 4 n bytes of the
//      device LLR arena (with a pinned staging twin), released when its request
//      completes, and 4 n bytes of the pinned result arena, released when the
//      caller collects the result.  The budget covers the whole device footprint:
//      each launch slot owns a fixed scratch region (queue counter, per-frame
//      metadata, the persistent forms' per-workgroup buffers), sized at creation
//      for the codes served and carved from the budget, and the LLR arena gets the
//      rest, so the dispatcher never allocates device memory;
//   3. launches: for every free launch slot (stream + workspace + flag arrays), the
//      code whose admitted work is oldest gets a batch of up to max_batch_frames of
//      its admitted frames: LLRs are copied into HBM on the slot's stream and one
//      persistent decode kernel runs them, writing x straight to pinned memory.
// Requests that arrive while others decode are therefore admitted as soon as
// memory frees up and start on the next free stream, overlapping on the device
// with the launches already running.  A frame's arithmetic depends only on its
// code's layout plan, so results are identical alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lpdec.h"
#include "lpdec_internal.h"
#include "lpdec_runtime.h"

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, capacity) (units: floats).
class RegionAllocator {
   public:
    explicit RegionAllocator(int64_t cap) : cap_(cap) { free_[0] = cap; }
    int64_t alloc(int64_t len) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                const int64_t off = it->first, rest = it->second - len;
                free_.erase(it);
                if (rest > 0) free_[off + len] = rest;
                used_ += len;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t len) {
        used_ -= len;
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t used() const { return used_; }
    int64_t capacity() const { return cap_; }

   private:
    int64_t cap_, used_ = 0;
    std::map<int64_t, int64_t> free_;
};

struct Request {
    int64_t ticket = 0;
    int code = 0, frames = 0, n = 0;
    int state = LPDEC_REQ_QUEUED;
    std::vector<float> llr;  // host copy until admission
    int64_t region = -1;     // offset (floats) in the LLR arenas (device + staging)
    int64_t xregion = -1;    // offset (floats) in the result arena, held until collected
    int launched = 0, finished = 0;
    std::vector<int32_t> iters;
    std::vector<uint8_t> flags;
    Clock::time_point t_submit, t_done;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    ScratchArena scratch{};  // this slot's device scratch (and pinned metadata staging)
    int *done = nullptr;       // pinned [cap]
    int32_t *iters = nullptr;  // pinned [cap]
    uint8_t *flags = nullptr;  // pinned [cap]
    std::vector<std::pair<Request *, int>> frames;
    std::vector<char> seen;
    std::vector<int64_t> llr_off, x_off;
    int code = -1, remaining = 0;
    bool busy = false;
};

}  // namespace

struct lpdec_server {
    std::vector<const lpdec_code *> codes;
    std::vector<int> n;
    lpdec_params params{};
    lpdec_server_config cfg{};
    bool gpu = true;

    float *d_llr = nullptr;  // device arena
    char *d_scratch = nullptr;  // the launch slots' scratch regions (one allocation)
    int64_t slot_scratch = 0;   // bytes of scratch per slot
    float *h_llr = nullptr;  // pinned staging arena
    float *h_x = nullptr;    // pinned result arena
    std::vector<float> null_llr, null_x;
    std::unique_ptr<RegionAllocator> regions;   // LLR arenas: the device budget
    std::unique_ptr<RegionAllocator> xregions;  // pinned result arena
    int64_t peak_bytes = 0;
    int peak_launches = 0;  // launch slots busy at once, at most

    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread th;
    bool stop = false;
    uint64_t gen = 0;  // bumped by every event that may unblock admission
    std::string thread_error;

    int64_t next_ticket = 1;
    std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
    std::deque<Request *> queue;                  // submitted, not admitted (FIFO)
    std::vector<std::deque<Request *>> admitted;  // per code, admitted with frames to launch
    std::vector<double> latencies;
    int64_t submitted = 0, completed = 0, cancelled = 0, rejected = 0, frames_done = 0, bits_done = 0,
            launches = 0;
    bool any_submit = false;
    Clock::time_point t_first, t_last;

    void run();
    bool collect();
    void admit();
    bool launch_into(Slot &s);
    void finish_frame(Request *r, int k, int32_t it, uint8_t fl);
};

void lpdec_server::finish_frame(Request *r, int k, int32_t it, uint8_t fl) {
    r->iters[k] = it;
    r->flags[k] = fl;
    if (++r->finished == r->frames) {
        r->state = LPDEC_REQ_DONE;
        r->t_done = Clock::now();
        t_last = r->t_done;
        regions->release(r->region, (int64_t)r->frames * r->n);
        latencies.push_back(std::chrono::duration<double>(r->t_done - r->t_submit).count());
        ++completed;
        frames_done += r->frames;
        bits_done += (int64_t)r->frames * r->n;
    }
}

// Scan running launches for finished frames.  Returns true if anything changed.
bool lpdec_server::collect() {
    bool changed = false;
    for (Slot &s : slots) {
        if (!s.busy) continue;
        for (size_t f = 0; f < s.frames.size(); ++f) {
            if (s.seen[f]) continue;
            const int d = __atomic_load_n(s.done + f, __ATOMIC_ACQUIRE);
            if (!d) continue;
            s.seen[f] = 1;
            --s.remaining;
            finish_frame(s.frames[f].first, s.frames[f].second, s.iters[f], s.flags[f]);
            changed = true;
        }
        if (s.remaining > 0 && gpu) {
            const hipError_t q = hipEventQuery(s.ev);
            if (q != hipErrorNotReady) {
                // The launch is over (or failed) but some frames never raised their
                // flag: rescan once, then fail the rest as not decoded.
                for (size_t f = 0; f < s.frames.size(); ++f) {
                    if (s.seen[f]) continue;
                    const bool ok = q == hipSuccess && __atomic_load_n(s.done + f, __ATOMIC_ACQUIRE);
                    if (!ok && thread_error.empty()) thread_error = "a launch ended without completing its frames";
                    s.seen[f] = 1;
                    --s.remaining;
                    finish_frame(s.frames[f].first, s.frames[f].second, ok ? s.iters[f] : 0,
                                 ok ? s.flags[f] : (uint8_t)0x80);
                }
                changed = true;
            }
        }
        if (s.remaining == 0 && (!gpu || hipEventQuery(s.ev) != hipErrorNotReady)) {
            s.busy = false;
            s.frames.clear();
            changed = true;
        }
    }
    if (changed) cv_done.notify_all();
    return changed;
}

void lpdec_server::admit() {
    while (!queue.empty()) {
        Request *r = queue.front();
        const int64_t len = (int64_t)r->frames * r->n;
        const int64_t off = regions->alloc(len);
        if (off < 0) break;  // wait for memory: later requests may not overtake
        const int64_t xoff = xregions->alloc(len);
        if (xoff < 0) {  // results not yet collected hold the result arena
            regions->release(off, len);
            break;
        }
        r->region = off;
        r->xregion = xoff;
        float *dst = gpu ? h_llr + off : null_llr.data() + off;
        std::memcpy(dst, r->llr.data(), sizeof(float) * len);
        std::vector<float>().swap(r->llr);
        r->state = LPDEC_REQ_RUNNING;
        admitted[r->code].push_back(r);
        queue.pop_front();
        peak_bytes = std::max(peak_bytes, regions->used() * (int64_t)sizeof(float));
    }
}

bool lpdec_server::launch_into(Slot &s) {
    // the code whose oldest admitted request is oldest
    int best = -1;
    for (size_t c = 0; c < admitted.size(); ++c) {
        if (admitted[c].empty()) continue;
        if (best < 0 || admitted[c].front()->ticket < admitted[best].front()->ticket) best = (int)c;
    }
    if (best < 0) return false;
    s.frames.clear();
    s.llr_off.clear();
    s.x_off.clear();
    auto &q = admitted[best];
    const int n = this->n[best];
    while (!q.empty() && (int)s.frames.size() < cfg.max_batch_frames) {
        Request *r = q.front();
        const int take = std::min(r->frames - r->launched, cfg.max_batch_frames - (int)s.frames.size());
        for (int k = 0; k < take; ++k) {
            const int fk = r->launched + k;
            s.frames.emplace_back(r, fk);
            s.llr_off.push_back(r->region + (int64_t)fk * n);
            s.x_off.push_back(r->xregion + (int64_t)fk * n);
        }
        if (gpu) {
            const int64_t off = r->region + (int64_t)r->launched * n;
            hipError_t e = hipMemcpyAsync(d_llr + off, h_llr + off, sizeof(float) * take * n, hipMemcpyHostToDevice,
                                          s.stream);
            if (e != hipSuccess) thread_error = hipGetErrorString(e);
        }
        r->launched += take;
        if (r->launched == r->frames) q.pop_front();
    }
    const int nf = (int)s.frames.size();
    s.seen.assign(nf, 0);
    s.remaining = nf;
    s.code = best;
    s.busy = true;
    ++launches;
    if (!gpu) {
        for (int f = 0; f < nf; ++f) {
            std::fill_n(null_x.data() + s.x_off[f], n, 0.5f);
            s.iters[f] = 0;
            s.flags[f] = 0;
            __atomic_store_n(s.done + f, 1, __ATOMIC_RELEASE);
        }
        return true;
    }
    std::memset(s.done, 0, sizeof(int) * nf);
    const lpdec_code *code = codes[best];
    lpdec_status st = lpdec_decode_core(&code, 1, nf, nullptr, s.llr_off.data(), s.x_off.data(), d_llr, &params, h_x,
                                        s.iters, s.flags, nullptr, nullptr, 0, s.stream, nullptr, s.done,
                                        &s.scratch);
    if (st != LPDEC_OK) thread_error = lpdec_last_error();
    hipError_t e = hipEventRecord(s.ev, s.stream);
    if (e != hipSuccess) thread_error = hipGetErrorString(e);
    if (st != LPDEC_OK) {
        // the launch failed: report the frames as not decoded rather than hang
        for (int f = 0; f < nf; ++f) {
            std::fill_n(h_x + s.x_off[f], n, 0.5f);
            s.iters[f] = 0;
            s.flags[f] = 0x80;
            s.done[f] = 1;
        }
    }
    return true;
}

void lpdec_server::run() {
    if (gpu) (void)hipSetDevice(codes[0]->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        collect();
        admit();
        for (Slot &s : slots)
            if (!s.busy && !launch_into(s)) break;
        bool busy = false;
        int nbusy = 0;
        for (Slot &s : slots) {
            busy |= s.busy;
            nbusy += s.busy;
        }
        peak_launches = std::max(peak_launches, nbusy);
        if (stop && !busy) break;
        if (busy) {
            cv_work.wait_for(lk, std::chrono::microseconds(20));
        } else {
            const uint64_t g = gen;  // nothing running: sleep until something changes
            cv_work.wait(lk, [&] { return stop || gen != g; });
        }
    }
}

extern "C" {

lpdec_server_config lpdec_server_default_config(void) {
    lpdec_server_config c;
    c.budget_bytes = (int64_t)256 << 20;
    c.max_batch_frames = 4096;
    c.max_inflight = 8;
    c.max_pending = 1 << 16;
    c.executor = LPDEC_EXECUTOR_GPU;
    return c;
}

lpdec_status lpdec_server_create(const lpdec_code *const *codes, const int32_t *code_n, int32_t ncodes,
                                 const lpdec_params *p, const lpdec_server_config *cfg_in, lpdec_server **out) {
    if (!out) return lpdec_fail(LPDEC_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (ncodes < 1) return lpdec_fail(LPDEC_EINVAL, "ncodes must be >= 1");
    lpdec_server_config cfg = cfg_in ? *cfg_in : lpdec_server_default_config();
    if (cfg.budget_bytes <= 0) return lpdec_fail(LPDEC_EINVAL, "budget_bytes must be > 0");
    if (cfg.max_batch_frames < 1) return lpdec_fail(LPDEC_EINVAL, "max_batch_frames must be >= 1");
    if (cfg.max_inflight < 1 || cfg.max_inflight > 8) return lpdec_fail(LPDEC_EINVAL, "max_inflight must be 1..8");
    if (cfg.max_pending < 1) return lpdec_fail(LPDEC_EINVAL, "max_pending must be >= 1");
    if (cfg.executor != LPDEC_EXECUTOR_GPU && cfg.executor != LPDEC_EXECUTOR_HOST_NULL)
        return lpdec_fail(LPDEC_EINVAL, "unknown executor %d", cfg.executor);
    const bool gpu = cfg.executor == LPDEC_EXECUTOR_GPU;
    std::unique_ptr<lpdec_server> s(new (std::nothrow) lpdec_server());
    if (!s) return lpdec_fail(LPDEC_ENOMEM, "host allocation failed");
    s->gpu = gpu;
    s->cfg = cfg;
    s->params = p ? *p : lpdec_default_params();
    if (s->params.storage != LPDEC_STORAGE_FP32 || s->params.mode == LPDEC_MODE_STREAMED)
        return lpdec_fail(LPDEC_EUNSUPPORTED, "the server runs the persistent FP32 forms");
    for (int c = 0; c < ncodes; ++c) {
        int n = 0;
        if (codes) {
            if (!codes[c]) return lpdec_fail(LPDEC_EINVAL, "codes[%d] is NULL", c);
            lpdec_code_info info;
            lpdec_status st = lpdec_code_get_info(codes[c], &info);
            if (st != LPDEC_OK) return st;
            n = info.n;
            s->codes.push_back(codes[c]);
        } else {
            if (gpu) return lpdec_fail(LPDEC_EINVAL, "the GPU executor needs code handles");
            if (!code_n || code_n[c] < 1) return lpdec_fail(LPDEC_EINVAL, "code_n[%d] must be >= 1", c);
            n = code_n[c];
        }
        s->n.push_back(n);
    }
    // Launch-slot scratch: enough for a launch of max_batch_frames frames of any
    // served code at its full persistent grid, but at most half the budget over all
    // slots (a slot then runs fewer workgroups at once; results do not depend on
    // the grid), and never less than one workgroup of the most demanding code.
    int64_t need_full = 0, need_min = 0, host_meta = 0, nmin = INT64_MAX;
    for (int c = 0; c < ncodes; ++c) nmin = std::min<int64_t>(nmin, s->n[c]);
    if (gpu) {
        for (int c = 0; c < ncodes; ++c) {
            ScratchNeed sn;
            lpdec_status st = lpdec_scratch_need(codes[c], &s->params, cfg.max_batch_frames, true, &sn);
            if (st != LPDEC_OK) return st;
            if (sn.streamed) return lpdec_fail(LPDEC_EUNSUPPORTED, "the server runs the persistent FP32 forms");
            need_full = std::max<int64_t>(need_full, (int64_t)(sn.fixed + sn.per_wg * (size_t)sn.grid));
            need_min = std::max<int64_t>(need_min, (int64_t)(sn.fixed + sn.per_wg));
            host_meta = std::max<int64_t>(host_meta, (int64_t)sn.host);
        }
        const int64_t cap_share = cfg.budget_bytes / (2 * (int64_t)cfg.max_inflight);
        int64_t per = std::min(need_full, std::max(need_min, cap_share));
        per = (per + 255) / 256 * 256;
        s->slot_scratch = per;
    }
    const int64_t scratch_total = s->slot_scratch * cfg.max_inflight;
    if (cfg.budget_bytes - scratch_total < (int64_t)sizeof(float) * nmin)
        return lpdec_fail(LPDEC_EINVAL,
                          "budget of %lld bytes is too small: the launch slots' scratch takes %lld bytes and one "
                          "frame of the shortest code needs %lld more",
                          (long long)cfg.budget_bytes, (long long)scratch_total, (long long)(sizeof(float) * nmin));
    const int64_t cap = (cfg.budget_bytes - scratch_total) / (int64_t)sizeof(float);
    s->regions.reset(new RegionAllocator(cap));
    s->xregions.reset(new RegionAllocator(cap));
    s->admitted.resize(ncodes);
    const int ncap = cfg.max_batch_frames;
    s->slots.resize(cfg.max_inflight);
    if (gpu) {
        hipError_t e;
        if ((e = hipMalloc(&s->d_llr, sizeof(float) * cap)) != hipSuccess)
            return lpdec_fail(LPDEC_ENOMEM, "device arena of %lld bytes: %s", (long long)(sizeof(float) * cap),
                              hipGetErrorString(e));
        if ((e = hipMalloc(reinterpret_cast<void **>(&s->d_scratch), (size_t)scratch_total)) != hipSuccess)
            return lpdec_fail(LPDEC_ENOMEM, "launch scratch of %lld bytes: %s", (long long)scratch_total,
                              hipGetErrorString(e));
        const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&s->h_llr), sizeof(float) * cap, hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void **>(&s->h_x), sizeof(float) * cap, fl)) != hipSuccess)
            return lpdec_fail(LPDEC_ENOMEM, "pinned arenas: %s", hipGetErrorString(e));
        for (Slot &sl : s->slots) {
            if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming)) != hipSuccess ||
                (e = hipHostMalloc(reinterpret_cast<void **>(&sl.done), sizeof(int) * ncap, fl)) != hipSuccess ||
                (e = hipHostMalloc(reinterpret_cast<void **>(&sl.iters), sizeof(int32_t) * ncap, fl)) != hipSuccess ||
                (e = hipHostMalloc(reinterpret_cast<void **>(&sl.flags), ncap, fl)) != hipSuccess ||
                (e = hipHostMalloc(reinterpret_cast<void **>(&sl.scratch.host), (size_t)host_meta,
                                   hipHostMallocDefault)) != hipSuccess)
                return lpdec_fail(LPDEC_EDEVICE, "launch slot set-up: %s", hipGetErrorString(e));
            sl.scratch.base = s->d_scratch + (&sl - s->slots.data()) * s->slot_scratch;
            sl.scratch.bytes = (size_t)s->slot_scratch;
            sl.scratch.host_bytes = (size_t)host_meta;
        }
    } else {
        s->null_llr.assign(cap, 0.0f);
        s->null_x.assign(cap, 0.0f);
        for (Slot &sl : s->slots) {
            sl.done = new int[ncap];
            sl.iters = new int32_t[ncap];
            sl.flags = new uint8_t[ncap];
        }
    }
    lpdec_server *raw = s.get();
    s->th = std::thread([raw] { raw->run(); });
    *out = s.release();
    return LPDEC_OK;
}

lpdec_status lpdec_server_submit(lpdec_server *s, int32_t code, int32_t frames, const float *llr, int64_t *ticket) {
    if (!s || !ticket) return lpdec_fail(LPDEC_EINVAL, "server and ticket must not be NULL");
    if (code < 0 || code >= (int)s->n.size()) return lpdec_fail(LPDEC_EINVAL, "code index %d out of range", code);
    if (frames < 1) return lpdec_fail(LPDEC_EINVAL, "frames must be >= 1");
    if (!llr) return lpdec_fail(LPDEC_EINVAL, "llr must not be NULL");
    const int n = s->n[code];
    const int64_t bytes = (int64_t)frames * n * (int64_t)sizeof(float);
    std::unique_ptr<Request> r(new Request());
    r->code = code;
    r->frames = frames;
    r->n = n;
    r->llr.assign(llr, llr + (size_t)frames * n);
    r->iters.assign(frames, 0);
    r->flags.assign(frames, 0);
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t arena = s->regions->capacity() * (int64_t)sizeof(float);
    if (bytes > arena) {
        ++s->rejected;
        return lpdec_fail(LPDEC_EINVAL,
                          "request of %lld bytes exceeds the server budget of %lld bytes (%lld bytes of LLR arena "
                          "beside the launch slots' scratch)",
                          (long long)bytes, (long long)s->cfg.budget_bytes, (long long)arena);
    }
    if ((int)s->queue.size() >= s->cfg.max_pending) {
        ++s->rejected;
        return lpdec_fail(LPDEC_EBUSY, "%d requests already queued", (int)s->queue.size());
    }
    if (!s->thread_error.empty()) return lpdec_fail(LPDEC_EDEVICE, "server failed: %s", s->thread_error.c_str());
    r->ticket = s->next_ticket++;
    r->t_submit = Clock::now();
    if (!s->any_submit) {
        s->any_submit = true;
        s->t_first = r->t_submit;
    }
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->reqs.emplace(r->ticket, std::move(r));
    ++s->submitted;
    ++s->gen;
    s->cv_work.notify_one();
    return LPDEC_OK;
}

lpdec_status lpdec_server_poll(lpdec_server *s, int64_t ticket, int32_t *state) {
    if (!s || !state) return lpdec_fail(LPDEC_EINVAL, "server and state must not be NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return lpdec_fail(LPDEC_EINVAL, "unknown ticket %lld", (long long)ticket);
    *state = it->second->state;
    return LPDEC_OK;
}

lpdec_status lpdec_server_wait(lpdec_server *s, int64_t ticket, double timeout_s, float *x, int32_t *iters,
                               uint8_t *flags, double *latency_s) {
    if (!s) return lpdec_fail(LPDEC_EINVAL, "server must not be NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return lpdec_fail(LPDEC_EINVAL, "unknown ticket %lld", (long long)ticket);
    Request *r = it->second.get();
    auto ready = [&] { return r->state == LPDEC_REQ_DONE || !s->thread_error.empty(); };
    if (timeout_s < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
        return lpdec_fail(LPDEC_EBUSY, "request %lld not finished within %.3f s", (long long)ticket, timeout_s);
    if (r->state != LPDEC_REQ_DONE) return lpdec_fail(LPDEC_EDEVICE, "server failed: %s", s->thread_error.c_str());
    const size_t len = (size_t)r->frames * r->n;
    if (x) {
        const float *src = s->gpu ? s->h_x + r->xregion : s->null_x.data() + r->xregion;
        std::memcpy(x, src, sizeof(float) * len);
    }
    s->xregions->release(r->xregion, (int64_t)len);
    ++s->gen;
    s->cv_work.notify_one();  // a queued request may fit now
    if (iters) std::memcpy(iters, r->iters.data(), sizeof(int32_t) * r->frames);
    if (flags) std::memcpy(flags, r->flags.data(), r->frames);
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    s->reqs.erase(it);
    return LPDEC_OK;
}

lpdec_status lpdec_server_cancel(lpdec_server *s, int64_t ticket) {
    if (!s) return lpdec_fail(LPDEC_EINVAL, "server must not be NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return lpdec_fail(LPDEC_EINVAL, "unknown ticket %lld", (long long)ticket);
    if (it->second->state != LPDEC_REQ_QUEUED)
        return lpdec_fail(LPDEC_EBUSY, "request %lld is already admitted", (long long)ticket);
    auto q = std::find(s->queue.begin(), s->queue.end(), it->second.get());
    if (q != s->queue.end()) s->queue.erase(q);
    s->reqs.erase(it);
    ++s->cancelled;
    ++s->gen;
    s->cv_work.notify_one();
    return LPDEC_OK;
}

lpdec_status lpdec_server_get_stats(lpdec_server *s, lpdec_server_stats *st) {
    if (!s || !st) return lpdec_fail(LPDEC_EINVAL, "server and stats must not be NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(st, 0, sizeof *st);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->cancelled = s->cancelled;
    st->rejected = s->rejected;
    st->frames_completed = s->frames_done;
    st->bits_completed = s->bits_done;
    st->inflight_bytes = s->regions->used() * (int64_t)sizeof(float);
    st->peak_bytes = s->peak_bytes;
    st->workspace_bytes = s->slot_scratch * (int64_t)s->slots.size();
    st->peak_device_bytes = st->workspace_bytes + s->peak_bytes;
    st->peak_concurrent_launches = s->peak_launches;
    st->launches = s->launches;
    st->queued = (int32_t)s->queue.size();
    int running = 0;
    for (auto &kv : s->reqs) running += kv.second->state == LPDEC_REQ_RUNNING;
    st->running = running;
    if (!s->latencies.empty()) {
        std::vector<double> l = s->latencies;
        std::sort(l.begin(), l.end());
        auto q = [&](double f) { return l[std::min(l.size() - 1, (size_t)(f * (l.size() - 1) + 0.5))]; };
        st->p50_latency_s = q(0.50);
        st->p99_latency_s = q(0.99);
        double sum = 0;
        for (double v : l) sum += v;
        st->mean_latency_s = sum / l.size();
        st->max_latency_s = l.back();
        st->elapsed_s = std::chrono::duration<double>(s->t_last - s->t_first).count();
    }
    return LPDEC_OK;
}

void lpdec_server_destroy(lpdec_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->queue.clear();  // queued requests are dropped; running launches finish
        s->cv_work.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    for (Slot &sl : s->slots) {
        if (s->gpu) {
            if (sl.stream) (void)hipStreamSynchronize(sl.stream);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
            if (sl.scratch.host) (void)hipHostFree(sl.scratch.host);
            if (sl.ev) (void)hipEventDestroy(sl.ev);
            if (sl.done) (void)hipHostFree(sl.done);
            if (sl.iters) (void)hipHostFree(sl.iters);
            if (sl.flags) (void)hipHostFree(sl.flags);
        } else {
            delete[] sl.done;
            delete[] sl.iters;
            delete[] sl.flags;
        }
    }
    if (s->d_llr) (void)hipFree(s->d_llr);
    if (s->d_scratch) (void)hipFree(s->d_scratch);
    if (s->h_llr) (void)hipHostFree(s->h_llr);
    if (s->h_x) (void)hipHostFree(s->h_x);
    delete s;
}

}  // extern "C"
