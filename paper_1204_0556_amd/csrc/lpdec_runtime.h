// Host-side runtime types shared by the decoder entry points (lpdec_host.cpp)
// and the serving loop (lpdec_server.cpp).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/lpdec.h"
#include "lpdec_internal.h"

// Reusable device buffer that only grows.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need) {
        if (need <= bytes) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            bytes = 0;
        }
        need = std::max<size_t>(need, 256);
        hipError_t e = hipMalloc(&p, need);
        if (e == hipSuccess) bytes = need;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};


// Workspace for one decode call; serialised across streams with an event.
struct Workspace {
    std::mutex mu;
    hipEvent_t last = nullptr;
    DevBuf queue;      // persistent work counter
    DevBuf codes;      // DevCode array (multi-code launches)
    DevBuf frame_meta; // code_of_frame / offsets
    DevBuf z, u, st, active, gslots, gstate, gmu, gxprev;
    DevBuf alist, alist_cnt;  // streamed form: the unfinished frames of the last launch
    int *host_active = nullptr; // pinned
    char *host_meta = nullptr;  // pinned staging for per-call metadata
    size_t host_meta_bytes = 0;
    // streamed form replayed from a graph: the device launch index, the capture
    // stream, and the instantiated block of launches with the arguments it holds
    DevBuf launch_dev;
    hipStream_t capture = nullptr;
    hipGraphExec_t graph = nullptr;
    std::vector<char> graph_key;
    ~Workspace() {
        queue.release(); codes.release(); frame_meta.release();
        z.release(); u.release(); st.release(); active.release(); gslots.release(); gstate.release();
        gmu.release(); gxprev.release(); launch_dev.release(); alist.release(); alist_cnt.release();
        if (graph) (void)hipGraphExecDestroy(graph);
        if (capture) (void)hipStreamDestroy(capture);
        if (host_active) (void)hipHostFree(host_active);
        if (host_meta) (void)hipHostFree(host_meta);
        if (last) (void)hipEventDestroy(last);
    }
};

// Exclusive use of a workspace by one call: the call's stream first waits for
// the previous user's work, and the destructor records this call's completion.
struct WsGuard {
    Workspace &ws;
    hipStream_t stream;
    std::unique_lock<std::mutex> lk;
    WsGuard(Workspace &w, hipStream_t s) : ws(w), stream(s), lk(w.mu) {
        if (ws.last) (void)hipStreamWaitEvent(stream, ws.last, 0);
    }
    ~WsGuard() { (void)done(); }
    hipError_t done() {
        if (!ws.last) {
            hipError_t e = hipEventCreateWithFlags(&ws.last, hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        return hipEventRecord(ws.last, stream);
    }
};

struct lpdec_code {
    lpdec::DevCode dc{};   // host copy with device pointers
    lpdec::DevCode *d_dc = nullptr;
    std::vector<void *> allocs;
    int device = -1;
    bool resident_ok = false;
    lpdec::LaunchConfig resident_cfg{};
    int tune_bpc[3] = {0, 0, 0};     // workgroups per CU by form (0: runtime estimate)
    int tune_variant[3] = {-1, -1, -1};  // kernel variant by form (streamed only; -1: default)
    // multi-code launches led by this code: hand out frames of larger codes first
    // (1), in submission order (0), or the default (-1: larger first when sizes differ)
    int tune_order = -1;
    bool graph = false;  // streamed form: replay each block of launches from a captured graph
    Workspace ws;
    ~lpdec_code() {
        if (d_dc) (void)hipFree(d_dc);
        for (void *p : allocs) (void)hipFree(p);
    }
};


// Sets the thread-local message returned by lpdec_last_error() and returns st.
lpdec_status lpdec_fail(lpdec_status st, const char *fmt, ...);

// Device scratch lent by the caller of a decode that must not allocate: the
// queue counter and every per-workgroup buffer of the persistent forms are carved
// out of it, and the persistent grid is cut to what it holds (results do not
// depend on the grid).  No workspace, event or lock of the code is touched.
struct ScratchArena {
    char *base;    // device address, 256-byte aligned
    size_t bytes;  // capacity
    // optional pinned host staging for per-frame metadata (scattered frames,
    // completion flags); the caller keeps the previous call on this arena finished
    // before the next one starts, so the staging is never overwritten in flight
    char *host = nullptr;
    size_t host_bytes = 0;
};

// Device scratch one decode launch needs: `fixed` bytes (queue counter and
// per-frame metadata) plus `per_wg` bytes for each persistent workgroup; `grid`
// is the grid the launch would use without a cap.  Each buffer is 256-byte
// aligned, so an arena of fixed + per_wg * g + 1024 bytes holds g workgroups.
struct ScratchNeed {
    size_t fixed = 0, per_wg = 0, host = 0;
    int grid = 0;
    bool streamed = false;  // the streamed form (per-frame state): no arena serves it
};
lpdec_status lpdec_scratch_need(const lpdec_code *code, const lpdec_params *p, int nframes, bool scattered,
                                ScratchNeed *out);

// Decode core shared by every entry point (see lpdec_host.cpp).
lpdec_status lpdec_decode_core(const lpdec_code *const *codes, int ncodes, int nframes,
                               const int32_t *code_of_frame, const int64_t *llr_off, const int64_t *x_off,
                               const float *llr, const lpdec_params *pin, float *x_out, int32_t *iters_out,
                               uint8_t *flags_out, float *z_state, float *u_state, int state_flags, void *stream_v,
                               Workspace *ws_in, int *done, const ScratchArena *arena = nullptr);
