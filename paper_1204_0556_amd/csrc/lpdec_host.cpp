// Host runtime of the MI355X ADMM LP decoder: code validation and layout
// planning, device upload, workspace management and the C ABI of lpdec.h.
//
// The layout plan (see DevCode in lpdec_internal.h) is what makes the kernels
// coalesced and register-resident:
//   * checks are grouped by degree into chunks of 64, one check per wave lane,
//     with edge state stored lane-minor inside a chunk;
//   * variables are renumbered by decreasing degree so that a variable's replicas
//     form one contiguous slot block (its CSC block), summed in a fixed order;
//   * chunk c belongs to wave c % waves, so a workgroup of `waves` wavefronts
//     covers one frame and each wave owns `cpt` chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/lpdec.h"
#include "lpdec_aux.h"
#include "lpdec_internal.h"
#include "lpdec_runtime.h"

using namespace lpdec;

static thread_local std::string g_last_error;

lpdec_status lpdec_fail(lpdec_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

namespace {

#define fail lpdec_fail

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            return fail(LPDEC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));        \
    } while (0)

// Device properties, queried once per device.
struct DeviceInfo {
    int device = -1;
    int cus = 0;
    size_t max_lds = 0;
};

DeviceInfo device_info() {
    DeviceInfo di;
    if (hipGetDevice(&di.device) != hipSuccess) return di;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, di.device) != hipSuccess) return di;
    di.cus = prop.multiProcessorCount;
    di.max_lds = prop.sharedMemPerBlock;
    // gfx950 exposes 160 KB of LDS per workgroup.
    if (prop.maxSharedMemoryPerMultiProcessor > di.max_lds) di.max_lds = prop.maxSharedMemoryPerMultiProcessor;
    return di;
}

template <typename T>
hipError_t upload(const std::vector<T> &h, T **d) {
    *d = nullptr;
    if (h.empty()) return hipSuccess;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(d), h.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// Validation and layout planning.

lpdec_status build_plan(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                        lpdec_code *code) {
    if (m < 1 || n < 1) return fail(LPDEC_EINVAL, "m and n must be >= 1 (got m=%d n=%d)", m, n);
    if (!row_ptr || !col_idx) return fail(LPDEC_EINVAL, "row_ptr and col_idx must not be NULL");
    if (nnz < 1 || row_ptr[0] != 0 || row_ptr[m] != nnz)
        return fail(LPDEC_EINVAL, "row_ptr must start at 0 and end at nnz=%lld", (long long)nnz);
    if (n > 65536 || nnz > 65536)
        return fail(LPDEC_EUNSUPPORTED, "codes with n > 65536 or nnz > 65536 are not supported (n=%d nnz=%lld)", n,
                    (long long)nnz);
    std::vector<int> vdeg(n, 0);
    int dmin = 1 << 30, dmax = 0;
    for (int j = 0; j < m; ++j) {
        const int d = row_ptr[j + 1] - row_ptr[j];
        if (d < 0) return fail(LPDEC_EINVAL, "row_ptr decreases at row %d", j);
        if (row_ptr[j + 1] > nnz) return fail(LPDEC_EINVAL, "row_ptr[%d] exceeds nnz", j + 1);
        if (d < 2) return fail(LPDEC_EINVAL, "row %d has degree %d; checks need degree >= 2", j, d);
        if (d > LPDEC_MAX_CHECK_DEGREE)
            return fail(LPDEC_EUNSUPPORTED, "row %d has degree %d > %d", j, d, LPDEC_MAX_CHECK_DEGREE);
        dmin = std::min(dmin, d);
        dmax = std::max(dmax, d);
        for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e) {
            const int c = col_idx[e];
            if (c < 0 || c >= n) return fail(LPDEC_EINVAL, "column index %d out of range in row %d", c, j);
            if (e > row_ptr[j] && c <= col_idx[e - 1])
                return fail(LPDEC_EINVAL, "row %d: column indices must be strictly increasing", j);
            vdeg[c]++;
        }
    }
    for (int i = 0; i < n; ++i)
        if (vdeg[i] == 0) return fail(LPDEC_EINVAL, "column %d has no checks (empty column of H)", i);

    // variables: stable order by decreasing degree
    std::vector<int> vorder(n);
    std::iota(vorder.begin(), vorder.end(), 0);
    std::stable_sort(vorder.begin(), vorder.end(), [&](int a, int b) { return vdeg[a] > vdeg[b]; });
    std::vector<int> vint(n);
    for (int i = 0; i < n; ++i) vint[vorder[i]] = i;
    DevCode &D = code->dc;
    D.m = m;
    D.n = n;
    D.E = (int)nnz;
    D.dmin = dmin;
    D.dmax = dmax;
    D.var_identity = 1;
    for (int i = 0; i < n; ++i)
        if (vorder[i] != i) D.var_identity = 0;
    // degree classes
    D.nvc = 0;
    int slot = 0;
    for (int i = 0; i < n; ++i) {
        const int d = vdeg[vorder[i]];
        if (D.nvc == 0 || D.vc_deg[D.nvc - 1] != d) {
            if (D.nvc == 8) return fail(LPDEC_EUNSUPPORTED, "more than 8 distinct variable degrees");
            D.vc_start[D.nvc] = i;
            D.vc_slot0[D.nvc] = slot;
            D.vc_deg[D.nvc] = d;
            D.vc_inv[D.nvc] = 1.0f / (float)d;
            D.nvc++;
        }
        slot += d;
    }
    D.dv = (D.nvc == 1) ? D.vc_deg[0] : 0;
    D.dv_inv = (D.nvc == 1) ? D.vc_inv[0] : 0.0f;
    std::vector<int2> vinfo(n);
    for (int c = 0; c < D.nvc; ++c) {
        const int end = (c + 1 < D.nvc) ? D.vc_start[c + 1] : n;
        for (int i = D.vc_start[c]; i < end; ++i) {
            vinfo[i].x = (D.vc_slot0[c] + (i - D.vc_start[c]) * D.vc_deg[c]) | (D.vc_deg[c] << 24);
            float inv = D.vc_inv[c];
            std::memcpy(&vinfo[i].y, &inv, sizeof inv);
        }
    }
    for (int c = D.nvc; c <= 8; ++c) D.vc_start[c] = n;
    for (int c = D.nvc; c < 8; ++c) {
        D.vc_slot0[c] = slot;
        D.vc_deg[c] = 1;
        D.vc_inv[c] = 1.0f;
    }
    // slot of every CSR edge: variable blocks in internal order, edges ascending
    std::vector<int> vstart(n + 1, 0);
    for (int i = 0; i < n; ++i) vstart[i + 1] = vstart[i] + vdeg[vorder[i]];
    std::vector<int> fill(vstart.begin(), vstart.end() - 1);
    std::vector<int> eslot(nnz);
    for (int j = 0; j < m; ++j)
        for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e) eslot[e] = fill[vint[col_idx[e]]]++;

    // checks grouped by degree (stable), chunks of 64
    std::vector<int> corder(m);
    std::iota(corder.begin(), corder.end(), 0);
    std::stable_sort(corder.begin(), corder.end(), [&](int a, int b) {
        return (row_ptr[a + 1] - row_ptr[a]) < (row_ptr[b + 1] - row_ptr[b]);
    });
    std::vector<int> chunk_deg, chunk_off, chunk_cnt;
    std::vector<uint32_t> meta;
    std::vector<int> ecsr;
    int pos = 0;
    while (pos < m) {
        const int d = row_ptr[corder[pos] + 1] - row_ptr[corder[pos]];
        int cnt = 0;
        while (pos + cnt < m && cnt < kWave && (row_ptr[corder[pos + cnt] + 1] - row_ptr[corder[pos + cnt]]) == d)
            ++cnt;
        const int off = (int)meta.size();
        chunk_deg.push_back(d);
        chunk_off.push_back(off);
        chunk_cnt.push_back(cnt);
        meta.resize(off + (size_t)d * kWave, 0u);
        ecsr.resize(off + (size_t)d * kWave, -1);
        for (int l = 0; l < cnt; ++l) {
            const int j = corder[pos + l];
            for (int k = 0; k < d; ++k) {
                const int e = row_ptr[j] + k;
                meta[off + k * kWave + l] = ((uint32_t)eslot[e] << 16) | (uint32_t)vint[col_idx[e]];
                ecsr[off + k * kWave + l] = e;
            }
        }
        pos += cnt;
    }
    D.nchunks = (int)chunk_deg.size();
    D.E_int = (int)meta.size();
    // waves: as many as possible up to 16 per workgroup (fewer chunks per wave),
    // except for codes with checks of degree 7..8 (all >= 6) that the resident
    // form can hold: those get at most 8 waves, so that up to 8 chunks per wave
    // fit in the 256 registers a wave has at 2 waves per SIMD (at 16 waves a
    // wave has 128, too few for 4 degree-8 chunks).  Every form of a code uses
    // the same plan, so the forms stay bitwise identical.
    const bool wide = dmin >= 6 && dmax > 6 && dmax <= 8 && D.nchunks <= 8 * 8 &&
                      4 * ((size_t)nnz + n) + 1024 <= 160 * 1024;
    const int max_waves = wide ? 8 : kMaxWaves;
    D.cpt = (D.nchunks + max_waves - 1) / max_waves;
    D.waves = (D.nchunks + D.cpt - 1) / D.cpt;

    // accumulator exchange: each edge's entry as a byte offset (8 bytes per variable),
    // so that the kernels address LDS without unpacking the metadata
    std::vector<uint32_t> acc_off(meta.size());
    for (size_t i = 0; i < meta.size(); ++i) acc_off[i] = 8u * (meta[i] & 0xffffu);
    int *d_cdeg, *d_coff, *d_ccnt, *d_ecsr, *d_vorig;
    uint32_t *d_meta, *d_acc;
    int2 *d_vinfo;
    hipError_t e = hipGetDevice(&code->device);
    if (e != hipSuccess) return fail(LPDEC_EDEVICE, "no HIP device: %s", hipGetErrorString(e));
    if ((e = upload(chunk_deg, &d_cdeg)) != hipSuccess ||
        (code->allocs.push_back(d_cdeg), (e = upload(chunk_off, &d_coff)) != hipSuccess) ||
        (code->allocs.push_back(d_coff), (e = upload(chunk_cnt, &d_ccnt)) != hipSuccess) ||
        (code->allocs.push_back(d_ccnt), (e = upload(meta, &d_meta)) != hipSuccess) ||
        (code->allocs.push_back(d_meta), (e = upload(acc_off, &d_acc)) != hipSuccess) ||
        (code->allocs.push_back(d_acc), (e = upload(ecsr, &d_ecsr)) != hipSuccess) ||
        (code->allocs.push_back(d_ecsr), (e = upload(vorder, &d_vorig)) != hipSuccess) ||
        (code->allocs.push_back(d_vorig), (e = upload(vinfo, &d_vinfo)) != hipSuccess))
        return fail(e == hipErrorOutOfMemory ? LPDEC_ENOMEM : LPDEC_EDEVICE, "uploading the code: %s",
                    hipGetErrorString(e));
    code->allocs.push_back(d_vinfo);
    D.var_info = d_vinfo;
    D.chunk_deg = d_cdeg;
    D.chunk_off = d_coff;
    D.chunk_cnt = d_ccnt;
    D.edge_meta = d_meta;
    D.edge_acc = d_acc;
    D.edge_csr = d_ecsr;
    D.var_orig = d_vorig;
    if ((e = hipMalloc(&code->d_dc, sizeof(DevCode))) != hipSuccess)
        return fail(LPDEC_ENOMEM, "allocating the code descriptor: %s", hipGetErrorString(e));
    if ((e = hipMemcpy(code->d_dc, &D, sizeof(DevCode), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(LPDEC_EDEVICE, "uploading the code descriptor: %s", hipGetErrorString(e));
    return LPDEC_OK;
}

// Launch-shape planning for a set of codes decoded together.
struct Shape {
    int ncodes = 0, nchunks = 0;
    int waves = 0, cpt = 0, nmax = 0, Emax = 0, Eint_max = 0, dclass = 0;
    int dv = 0;  // common variable degree of all codes (0 if mixed)
    int dreg = 0;  // common check degree of all codes (0 if mixed)
    bool permuted = false;  // some code renumbers its variables
};

Shape shape_of(const lpdec_code *const *codes, int ncodes) {
    Shape s;
    s.ncodes = ncodes;
    bool all6 = true, in68 = true, upto8 = true;
    for (int c = 0; c < ncodes; ++c) {
        const DevCode &D = codes[c]->dc;
        s.nchunks = std::max(s.nchunks, D.nchunks);
        s.waves = std::max(s.waves, D.waves);
        s.cpt = std::max(s.cpt, D.cpt);
        s.nmax = std::max(s.nmax, D.n);
        s.Emax = std::max(s.Emax, D.E);
        s.Eint_max = std::max(s.Eint_max, D.E_int);
        all6 = all6 && D.dmin == 6 && D.dmax == 6;
        in68 = in68 && D.dmin >= 6 && D.dmax <= 8;
        upto8 = upto8 && D.dmax <= 8;
        s.permuted = s.permuted || !D.var_identity;
    }
    s.dclass = all6 ? 0 : (in68 ? 2 : (upto8 ? 1 : 3));
    s.dv = (codes[0]->dc.nvc == 1) ? codes[0]->dc.vc_deg[0] : 0;
    for (int c = 1; c < ncodes; ++c)
        if (codes[c]->dc.nvc != 1 || codes[c]->dc.vc_deg[0] != s.dv) s.dv = 0;
    s.dreg = codes[0]->dc.dmin == codes[0]->dc.dmax ? codes[0]->dc.dmin : 0;
    for (int c = 1; c < ncodes; ++c)
        if (codes[c]->dc.dmin != s.dreg || codes[c]->dc.dmax != s.dreg) s.dreg = 0;
    return s;
}

constexpr size_t kStaticLds = 1024;  // s_red + s_frame + alignment
constexpr size_t kLdsLimit = 160 * 1024;

// Two frames per workgroup (k_decode_pair): the code's plan of W waves (wave v
// owns chunks v and v + W) becomes W virtual waves per frame, placed on 12
// physical waves with at most one virtual wave of each frame per physical wave.
// Wave p runs on SIMD p % 4 of its CU (waves are dealt to the SIMDs in turn), and
// the check phase lasts as long as the SIMD with the most chunks, so the virtual
// waves are placed largest first, each where its SIMD holds the fewest chunks so
// far (then the physical wave with the fewest, then the lowest index).  Returns
// the chunks of the busiest SIMD, or 0 if the plan does not fit.
int pair_plan(int nchunks, int W, unsigned long long host[2]) {
    constexpr int P = 12;
    if (W < 1 || W > P || nchunks > 2 * W) return 0;
    struct Item {
        int size, slot, v;
    };
    std::vector<Item> items;
    for (int slot = 0; slot < 2; ++slot)
        for (int v = 0; v < W; ++v) items.push_back({(v < nchunks) + (v + W < nchunks), slot, v});
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) { return a.size > b.size; });
    int hosted[P][2], load[P] = {0}, simd[4] = {0};
    for (int p = 0; p < P; ++p) hosted[p][0] = hosted[p][1] = -1;
    for (const Item &it : items) {
        int best = -1;
        for (int p = 0; p < P; ++p) {
            if (hosted[p][it.slot] >= 0) continue;
            if (best < 0 || simd[p % 4] < simd[best % 4] ||
                (simd[p % 4] == simd[best % 4] && load[p] < load[best]))
                best = p;
        }
        if (best < 0) return 0;
        hosted[best][it.slot] = it.v;
        load[best] += it.size;
        simd[best % 4] += it.size;
    }
    host[0] = host[1] = 0;
    for (int p = 0; p < P; ++p)
        for (int slot = 0; slot < 2; ++slot)
            host[slot] |= (unsigned long long)(hosted[p][slot] < 0 ? 0xF : hosted[p][slot]) << (4 * p);
    return *std::max_element(simd, simd + 4);
}

// Chunks of the busiest SIMD for one frame of a code planned with W waves of
// two chunks (wave v on SIMD v % 4).
int single_busiest(int nchunks, int W) {
    int simd[4] = {0};
    for (int v = 0; v < W; ++v) simd[v % 4] += (v < nchunks) + (v + W < nchunks);
    return *std::max_element(simd, simd + 4);
}

// Resident form: z,u in registers, slots and x in LDS.  Degree-6 codes: cpt <= 2
// chunks per wave with their metadata, gamma/mu of <= 8 variables per thread,
// <= 768 threads; one code whose variables all have degree 3 may run two frames
// per workgroup (variant 1; the default when it evens out the SIMDs' chunks);
// cpt 3..4 at up to 16 waves with the metadata and gamma/mu read from memory.
// Check degrees 6..8: cpt <= 8 chunks per wave, metadata and variable tables
// read from memory.
bool resident_config(const Shape &s, LaunchConfig *cfg, int variant = -1) {
    cfg->pair = false;
    if (s.dclass == 2) {
        // threads per template: cpt 1-2 up to 1024, cpt 4 up to 768, cpt 8 up to 512
        const int max_waves = s.cpt <= 2 ? kMaxWaves : (s.cpt <= 4 ? 12 : 8);
        if (s.cpt > 8 || s.waves > max_waves) return false;
        const size_t lds = 4 * ((size_t)s.Emax + s.nmax);
        if (lds + kStaticLds > kLdsLimit) return false;
        cfg->form = Form::Resident;
        cfg->cpt_tmpl = s.cpt <= 1 ? 1 : (s.cpt <= 2 ? 2 : (s.cpt <= 4 ? 4 : 8));
        cfg->vpt_tmpl = 0;
        cfg->dclass = 2;
        cfg->dv = 0;
        cfg->slot_mode = 1;
        cfg->half = false;
        cfg->threads = s.waves * kWave;
        cfg->lds_bytes = lds;
        cfg->lds_E = s.Emax;
        cfg->slot_stride = 0;
        cfg->state_stride = 0;
        return true;
    }
    if (s.dclass == 3) {
        // checks above degree 8: one chunk per wave, its z and u in registers
        const size_t lds = 4 * ((size_t)s.Emax + s.nmax);
        if (s.cpt > 1 || lds + kStaticLds > kLdsLimit) return false;
        cfg->form = Form::Resident;
        cfg->cpt_tmpl = 1;
        cfg->vpt_tmpl = 0;
        cfg->dclass = 3;
        cfg->dv = 0;
        cfg->slot_mode = 1;
        cfg->half = false;
        cfg->threads = s.waves * kWave;
        cfg->lds_bytes = lds;
        cfg->lds_E = s.Emax;
        cfg->slot_stride = 0;
        cfg->state_stride = 0;
        return true;
    }
    if (s.dclass != 0) return false;  // register budget only holds for degree-6 codes
    if (s.cpt > 4) return false;
    const int threads = s.waves * kWave;
    if (s.cpt > 2) {
        // three or four chunks per wave (codes up to 64 chunks, n up to about 8192 at
        // rate 1/2): up to 16 waves, z and u in registers, the edge metadata and
        // gamma/mu read from memory each iteration (the registers hold the state only)
        const size_t lds = 4 * ((size_t)s.Emax + s.nmax);
        if (threads > kMaxThreads || lds + kStaticLds > kLdsLimit) return false;
        cfg->form = Form::Resident;
        cfg->cpt_tmpl = 4;
        cfg->vpt_tmpl = 0;
        cfg->dclass = 0;
        cfg->dv = (s.dv == 3) ? 3 : 0;
        cfg->slot_mode = 1;
        cfg->half = false;
        cfg->threads = threads;
        cfg->lds_bytes = lds;
        cfg->lds_E = s.Emax;
        cfg->slot_stride = 0;
        cfg->state_stride = 0;
        return true;
    }
    if (threads > 768) return false;
    const int vpt = (s.nmax + threads - 1) / threads;
    if (vpt > 8) return false;
    const size_t lds = 4 * ((size_t)s.Emax + s.nmax);
    if (lds + kStaticLds > kLdsLimit) return false;
    cfg->form = Form::Resident;
    cfg->cpt_tmpl = (s.cpt <= 1 && vpt <= 4) ? 1 : 2;
    cfg->vpt_tmpl = vpt <= 4 ? 4 : 8;
    cfg->dclass = 0;
    cfg->dv = (s.dv == 3) ? 3 : 0;
    cfg->slot_mode = 1;
    cfg->half = false;
    cfg->threads = threads;
    cfg->lds_bytes = lds;
    cfg->lds_E = s.Emax;
    cfg->slot_stride = 0;
    cfg->state_stride = 0;
    // two frames per workgroup: one code, two chunks per wave, variables of degree 3,
    // <= 4 variables per thread of 12 waves; LDS holds each frame's slots and x
    unsigned long long host[2];
    const size_t pair_lds = 2 * lds;
    const bool pair_ok = variant != 0 && s.ncodes == 1 && s.cpt == 2 && s.dv == 3 && s.nmax <= 4 * 12 * kWave &&
                         pair_lds + kStaticLds <= kLdsLimit;
    const int busiest = pair_ok ? pair_plan(s.nchunks, s.waves, host) : 0;
    if (busiest > 0 && (variant >= 1 || busiest < 2 * single_busiest(s.nchunks, s.waves))) {
        cfg->pair = true;
        cfg->pair_host[0] = host[0];
        cfg->pair_host[1] = host[1];
        cfg->cpt_tmpl = 2;
        cfg->vpt_tmpl = 4;
        cfg->threads = 12 * kWave;
        cfg->lds_bytes = pair_lds;
    }
    return true;
}

// Large codes with the accumulator exchange whose checks all have degree 6 or 8
// may run k_decode_acc, which holds the first KR chunks of each wave in registers
// from phase A to phase C and walks the others one chunk ahead (KR = -1: k_decode,
// which walks every chunk without prefetch).  KR is bounded by the 128 registers a
// lane has at 16 waves per workgroup (the persistent-global form keeps its held
// chunks live across the whole iteration, so it holds fewer).  With FP16 storage
// the persistent-global form packs a held edge's z and u into one register and holds
// more: all of a wave's chunks (KR = kAccAllHeld, no walk) when the code has at most
// that many per wave.  FP32 persistent-global degree-6 codes of at most that many
// chunks per wave may also hold everything with two plan waves per hardware wave
// (returned as 2 kAccAllHeld: half the waves, twice the registers each).  variant < 0
// picks the default, else the variant-th candidate (clamped).  Returns KR.
int acc_held_chunks(const Shape &s, bool persistent, int variant, int *nvariants = nullptr, bool half = false) {
    static const int kStreamed6[] = {-1, 0, 2}, kStreamed8[] = {-1, 0, 2}, kPersist6[] = {-1, 0, 1, 2 * kAccAllHeld},
                     kPersist8[] = {-1, 0, 1}, kPersistHalf6[] = {kAccAllHeld, 4}, kPersistHalf8[] = {kAccAllHeld, 4};
    // defaults [persistent][degree 8] from the precision batches (8192 frames at
    // 2.5 dB): streamed (3,6) n = 16384 49.8 / 51.2 / 53.8 ms for KR = -1 / 0 / 2,
    // (4,8) 164.5 / 160.2 / 187.5 ms; persistent-global (3,6) 38.0 / 37.5 / 35.5 ms
    // for KR = -1 / 0 / 1, (4,8) 125.4 / 113.0 / 105.3 ms.  Since the streamed form's
    // per-launch frame lists, streamed (4,8) FP32 runs 141.3 / 140.2 / 136.3 ms for KR =
    // -1 / 0 / 2 and takes KR = 2, while FP16 storage keeps KR = 0 (114.2 / 110.7 / 144.0)
    static const int kDefault[2][2] = {{0, 1}, {2, 2}};
    const int *t = nullptr;
    int nt = 0;
    const bool ph = persistent && half;
    if (s.dreg == 6) {
        t = ph ? kPersistHalf6 : (persistent ? kPersist6 : kStreamed6);
        nt = ph ? (s.cpt <= kAccAllHeld ? 2 : 1) : 3;
        if (ph && s.cpt > kAccAllHeld) t = kPersistHalf6 + 1;
        if (persistent && !half && s.cpt <= kAccAllHeld && s.waves >= 2) nt = 4;
    } else if (s.dreg == 8) {
        t = ph ? kPersistHalf8 : (persistent ? kPersist8 : kStreamed8);
        nt = ph ? (s.cpt <= kAccAllHeld ? 2 : 1) : 3;
        if (ph && s.cpt > kAccAllHeld) t = kPersistHalf8 + 1;
    }
    if (nvariants) *nvariants = t && s.ncodes == 1 ? nt : 0;
    if (!t || s.ncodes != 1) return -1;
    // FP32 persistent-global degree 6: every chunk held at two plan waves per wave where
    // the code allows it ((3,6) n = 16384: 29.4 ms against 35.7 ms for one held chunk)
    const int def = ph ? 0
                       : (persistent && s.dreg == 6 && nt == 4
                              ? 3
                              : (!persistent && !half && s.dreg == 8 ? 2 : kDefault[persistent][s.dreg == 8]));
    const int v = variant < 0 ? def : std::min(variant, nt - 1);
    return t[v];
}

// Where the slot exchange of the non-resident forms lives: LDS float slots when
// 4 (E + n) bytes fit, else LDS fixed-point accumulators (8 n bytes), else global.
int slot_mode_for(const Shape &s, size_t *lds_bytes) {
    const size_t lds_slots = 4 * ((size_t)s.Emax + s.nmax), lds_acc = 8 * (size_t)s.nmax;
    if (lds_slots + kStaticLds <= kLdsLimit) { *lds_bytes = lds_slots; return 1; }
    if (lds_acc + kStaticLds <= kLdsLimit) { *lds_bytes = lds_acc; return 2; }
    *lds_bytes = 4 * (size_t)s.nmax;
    return 0;
}

// FP16 storage: only the accumulator kernel (large codes of check degree 6 or 8);
// returns false when the code has no such form.
bool persistent_global_config(const Shape &s, LaunchConfig *cfg, int variant = -1, bool half = false) {
    cfg->form = Form::PersistentGlobal;
    cfg->cpt_tmpl = 0;
    cfg->vpt_tmpl = 0;
    cfg->dclass = s.dclass == 2 ? 1 : s.dclass;
    cfg->dv = 0;
    cfg->slot_mode = slot_mode_for(s, &cfg->lds_bytes);
    cfg->half = half;
    cfg->threads = s.waves * kWave;
    cfg->lds_E = s.Emax;
    cfg->slot_stride = s.Emax;
    cfg->state_stride = s.Eint_max;
    cfg->acc_kr = cfg->slot_mode == 2 ? acc_held_chunks(s, true, variant, nullptr, half) : -1;
    cfg->acc = cfg->acc_kr >= 0;
    cfg->acc_d = cfg->acc ? s.dreg : 0;
    if (cfg->acc_kr == 2 * kAccAllHeld) cfg->threads = (s.waves + 1) / 2 * kWave;  // two plan waves per wave
    return !half || cfg->acc;
}

// Streamed variants (tuning value): 0 re-reads each chunk's z, u from HBM in every
// phase; 1 keeps two chunks per wave in registers, two workgroups per CU; 2 as 1
// with one workgroup per CU staging the next frame in LDS by direct-to-LDS loads
// (chosen only on request or by the autotuner).  Default: 1 when the code allows
// it, else 0.
void streamed_config(const Shape &s, bool half, LaunchConfig *cfg, int variant = -1) {
    cfg->form = Form::Streamed;
    cfg->slot_mode = slot_mode_for(s, &cfg->lds_bytes);
    cfg->cpt_tmpl = (cfg->slot_mode == 1 && s.cpt <= 2 && s.dclass == 0) ? 2 : 0;
    cfg->dclass = s.dclass == 2 ? 1 : s.dclass;
    const int threads = s.waves * kWave;
    // staged: all LDS static (z, u, slots of kStageEdges; gamma/mu, x of kStageVars)
    const size_t stage_lds = sizeof(float) * (3 * (size_t)kStageEdges + 2 * kStageVars);
    const bool stage_ok = cfg->cpt_tmpl == 2 && !half && threads <= 768 && s.dv > 0 &&
                          s.Eint_max <= kStageEdges && s.Emax <= kStageEdges && s.nmax <= kStageVars &&
                          s.nmax <= 4 * threads && stage_lds + kStaticLds <= kLdsLimit;
    if (variant == 0) cfg->cpt_tmpl = 0;
    cfg->staged = stage_ok && variant >= 2;
    if (cfg->staged) cfg->lds_bytes = 0;
    cfg->vpt_tmpl = 0;
    cfg->dv = 0;
    cfg->half = half;
    cfg->threads = s.waves * kWave;
    cfg->lds_E = s.Emax;
    cfg->slot_stride = s.Emax;
    cfg->state_stride = 0;
    cfg->acc_kr = cfg->slot_mode == 2 ? acc_held_chunks(s, false, variant, nullptr, half) : -1;
    cfg->acc = cfg->acc_kr >= 0;
    cfg->acc_d = cfg->acc ? s.dreg : 0;
}

// Workgroups of this configuration one compute unit can hold at once, from the
// kernel's registers, its LDS and its size: gfx950 has 4 SIMDs per CU, 512
// VGPRs per lane per SIMD (allocated in blocks of 8), at most 8 waves per SIMD
// and 160 KB of LDS per CU.
int resource_blocks_per_cu(const LaunchConfig &cfg, const KernelQuery &q) {
    const int waves = (cfg.threads + kWave - 1) / kWave;
    const int per_simd = (waves + 3) / 4;
    const int vg = std::max(8, (q.vgprs + 7) / 8 * 8);
    const int waves_per_simd = std::min(8, 512 / vg);
    int by_regs = waves_per_simd / per_simd;
    const size_t lds = cfg.lds_bytes + (size_t)q.static_lds;
    int by_lds = lds > 0 ? (int)((160 * 1024) / lds) : 32;
    return std::max(1, std::min(by_regs, by_lds));
}

// Workgroups per CU a launch uses: the code's tuned value for the form, else
// the runtime's occupancy estimate.
int blocks_per_cu(const LaunchConfig &cfg, const lpdec_code *code) {
    const int tuned = code ? code->tune_bpc[static_cast<int>(cfg.form)] : 0;
    if (tuned > 0) return tuned;
    KernelQuery q{};
    if (decode_query(cfg, &q) != hipSuccess || q.occupancy < 1) return 1;
    return q.occupancy;
}

int occupancy_grid(const LaunchConfig &cfg, int frames, const lpdec_code *code) {
    DeviceInfo di = device_info();
    const int cus = di.cus > 0 ? di.cus : 256;
    const int per_group = cfg.pair ? 2 : 1;  // frames a workgroup decodes at once
    return std::max(1, std::min((frames + per_group - 1) / per_group, cus * blocks_per_cu(cfg, code)));
}

lpdec_status check_params(const lpdec_params *p);

// Per-workgroup scratch of the persistent forms (bytes per workgroup; 0: unused):
// gamma/mu staged in internal variable order, the persistent-global state, the
// previous x of the accumulator exchange and the global slots.
struct WgBytes {
    size_t gmu = 0, state = 0, xprev = 0, slots = 0;
    size_t total() const { return gmu + state + xprev + slots; }
};
WgBytes wg_bytes(const Shape &s, const LaunchConfig &cfg) {
    WgBytes b;
    const bool pg = cfg.form == Form::PersistentGlobal;
    if (s.permuted && cfg.vpt_tmpl == 0) b.gmu = sizeof(float) * (size_t)s.nmax;
    if (pg) {
        b.state = 2 * (cfg.half ? 2 : sizeof(float)) * (size_t)cfg.state_stride;
        if (cfg.slot_mode == 2) b.xprev = sizeof(unsigned) * (size_t)s.nmax;
        if (cfg.slot_mode == 0) b.slots = sizeof(float) * (size_t)cfg.slot_stride;
    }
    return b;
}

// Host bytes of the per-frame metadata of a scattered single-code launch (code
// table, LLR and x offsets, code indices).
size_t meta_host_bytes(int nframes) {
    return ((sizeof(DevCode) + 255) / 256) * 256 + (size_t)nframes * (2 * sizeof(int64_t) + sizeof(int32_t));
}

// The form and launch configuration a decode of these codes with these
// parameters uses (the mode resolution of every decode entry point).
lpdec_status resolve_config(const Shape &s, const lpdec_params &p, bool scattered, LaunchConfig *cfg,
                            const lpdec_code *code) {
    const bool half = p.storage == LPDEC_STORAGE_FP16;
    int mode = p.mode;
    if (half && mode == LPDEC_MODE_RESIDENT)
        return fail(LPDEC_EUNSUPPORTED, "FP16 storage applies to the streamed and persistent-global forms");
    if (mode == LPDEC_MODE_AUTO && half) {
        // FP16: the persistent-global form where the code has it (its held chunks keep
        // the state in registers: faster than HBM round trips), else the streamed form
        LaunchConfig probe{};
        mode = persistent_global_config(s, &probe, -1, true) ? LPDEC_MODE_PERSISTENT_GLOBAL : LPDEC_MODE_STREAMED;
    }
    if (mode == LPDEC_MODE_AUTO) mode = LPDEC_MODE_RESIDENT;
    if (mode == LPDEC_MODE_RESIDENT &&
        !resident_config(s, cfg, code ? code->tune_variant[static_cast<int>(Form::Resident)] : -1)) {
        if (p.mode == LPDEC_MODE_RESIDENT)
            return fail(LPDEC_EUNSUPPORTED, "the register-resident form does not fit this code");
        mode = LPDEC_MODE_PERSISTENT_GLOBAL;
    }
    if (mode == LPDEC_MODE_PERSISTENT_GLOBAL &&
        !persistent_global_config(s, cfg, code ? code->tune_variant[static_cast<int>(Form::PersistentGlobal)] : -1,
                                  half))
        return fail(LPDEC_EUNSUPPORTED,
                    "FP16 storage in the persistent-global form needs one code whose checks all have degree 6 "
                    "or 8 and whose exchange uses the LDS accumulators (n too large for LDS slots)");
    if (mode == LPDEC_MODE_STREAMED) {
        if (scattered)
            return fail(LPDEC_EUNSUPPORTED, "the streamed form decodes one dense batch of one code per call");
        streamed_config(s, half, cfg, code ? code->tune_variant[static_cast<int>(Form::Streamed)] : -1);
        (void)code;
    }
    return LPDEC_OK;
}

lpdec_status check_params(const lpdec_params *p) {
    if (!(p->mu > 0.0f) || !std::isfinite(p->mu)) return fail(LPDEC_EINVAL, "mu must be a positive finite number");
    if (!(p->rho > 0.0f && p->rho < 2.0f)) return fail(LPDEC_EINVAL, "rho must lie in (0, 2)");
    if (p->max_iter < 1) return fail(LPDEC_EINVAL, "max_iter must be >= 1");
    if (!(p->tol >= 0.0f) || !std::isfinite(p->tol)) return fail(LPDEC_EINVAL, "tol must be finite and >= 0");
    if (p->storage != LPDEC_STORAGE_FP32 && p->storage != LPDEC_STORAGE_FP16)
        return fail(LPDEC_EINVAL, "unknown storage %d", p->storage);
    if (p->mode < LPDEC_MODE_AUTO || p->mode > LPDEC_MODE_PERSISTENT_GLOBAL)
        return fail(LPDEC_EINVAL, "unknown mode %d", p->mode);
    return LPDEC_OK;
}

// Acquire the workspace of the call's (first) code for exclusive use on `stream`.
}  // namespace

// Core decode over a set of codes.  With llr_off / x_off (host arrays) the frames
// are scattered in the llr / x buffers; code_of_frame (host) may be null when
// all frames use codes[0].  `ws` defaults to the first code's workspace; `done`
// (optional, host-visible) receives a completion flag per frame.
lpdec_status lpdec_decode_core(const lpdec_code *const *codes, int ncodes, int nframes,
                               const int32_t *code_of_frame, const int64_t *llr_off, const int64_t *x_off,
                               const float *llr, const lpdec_params *pin, float *x_out, int32_t *iters_out,
                               uint8_t *flags_out, float *z_state, float *u_state, int state_flags, void *stream_v,
                               Workspace *ws_in, int *done, const ScratchArena *arena) {
    lpdec_params p = pin ? *pin : lpdec_default_params();
    lpdec_status st = check_params(&p);
    if (st != LPDEC_OK) return st;
    if (nframes < 0) return fail(LPDEC_EINVAL, "batch must be >= 0");
    if (nframes == 0) return LPDEC_OK;
    if (!llr || !x_out || !iters_out || !flags_out)
        return fail(LPDEC_EINVAL, "llr, x_out, iters_out and flags_out must not be NULL");
    if ((z_state == nullptr) != (u_state == nullptr))
        return fail(LPDEC_EINVAL, "z_state and u_state must both be given or both be NULL");
    if (state_flags && !z_state) return fail(LPDEC_EINVAL, "state_flags given without state arrays");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    lpdec_code *c0 = const_cast<lpdec_code *>(codes[0]);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    for (int c = 0; c < ncodes; ++c)
        if (codes[c]->device != dev)
            return fail(LPDEC_EINVAL, "code %d was created on device %d, current device is %d", c, codes[c]->device,
                        dev);

    const Shape s = shape_of(codes, ncodes);
    LaunchConfig cfg{};
    const bool half = p.storage == LPDEC_STORAGE_FP16;
    st = resolve_config(s, p, ncodes > 1 || code_of_frame || llr_off || done, &cfg, codes[0]);
    if (st != LPDEC_OK) return st;
    if (arena && (ncodes > 1 || code_of_frame || ((llr_off || x_off || done) && !arena->host)))
        return fail(LPDEC_EINVAL, "lent scratch serves single-code batches (scattered ones with host staging)");
    if (arena && (cfg.form == Form::Streamed || half))
        return fail(LPDEC_EUNSUPPORTED,
                    "the allocation-free decode runs the persistent forms only (FP32 storage, mode AUTO, RESIDENT "
                    "or PERSISTENT_GLOBAL): the streamed form keeps every frame's state in HBM");
    // two frames per workgroup raise throughput only when every CU has two frames to
    // run; with fewer frames they would leave CUs idle and double each frame's time,
    // so the default keeps one frame per workgroup (an explicit variant 1 still pairs)
    if (cfg.pair && codes[0]->tune_variant[static_cast<int>(Form::Resident)] < 1) {
        const DeviceInfo di = device_info();
        if (nframes < 2 * (di.cus > 0 ? di.cus : 256)) resident_config(s, &cfg, 0);
    }

    Workspace &ws = ws_in ? *ws_in : c0->ws;
    // with lent scratch the code's workspace is not used, so it is neither locked
    // nor ordered after other calls (its event would be created on first use)
    std::unique_ptr<WsGuard> guard;
    if (!arena) guard.reset(new WsGuard(ws, stream));

    // per-launch code table and frame metadata
    const DevCode *codes_dev = c0->d_dc;
    FrameBatch fb{};
    fb.nframes = nframes;
    fb.llr = llr;
    fb.x_out = x_out;
    fb.iters_out = iters_out;
    fb.flags_out = flags_out;
    fb.done = done;
    size_t meta_bytes = 0;  // device bytes of the per-frame metadata (lent scratch: carved after the queue)
    if (ncodes > 1 || code_of_frame || llr_off) {
        // Metadata goes through pinned staging owned by the workspace.  The
        // previous call on this workspace may still be copying from it, so wait
        // for that call first (the source must outlive the asynchronous copy).
        // Lent scratch brings its own staging, which its owner keeps idle.
        const size_t tbl_bytes = ((sizeof(DevCode) * ncodes + 255) / 256) * 256;
        // frames of codes of different sizes are handed out largest code first, so
        // that the launch ends on short frames (less idle time in its tail); the
        // lookup costs a dependent load per frame, so equal-size codes skip it
        bool mixed_sizes = false;
        for (int c = 1; c < ncodes; ++c) mixed_sizes = mixed_sizes || codes[c]->dc.E != codes[0]->dc.E;
        const bool ordered = mixed_sizes && code_of_frame && codes[0]->tune_order != 0 &&
                             (cfg.form == Form::Resident || cfg.form == Form::PersistentGlobal);
        const size_t bytes = tbl_bytes + (size_t)nframes * (2 * sizeof(int64_t) + sizeof(int32_t)) +
                             (ordered ? (size_t)nframes * sizeof(int32_t) : 0);
        char *h, *d;
        meta_bytes = (bytes + 255) / 256 * 256;
        if (arena) {
            if (bytes > arena->host_bytes || 256 + meta_bytes > arena->bytes)
                return fail(LPDEC_EUNSUPPORTED, "per-frame metadata of %zu bytes exceeds the lent scratch", bytes);
            h = arena->host;
            d = arena->base + 256;
        } else {
            if (ws.last) HIP_TRY(hipEventSynchronize(ws.last));
            if (ws.host_meta_bytes < bytes) {
                if (ws.host_meta) HIP_TRY(hipHostFree(ws.host_meta));
                ws.host_meta = nullptr;
                ws.host_meta_bytes = 0;
                HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&ws.host_meta), bytes, hipHostMallocDefault));
                ws.host_meta_bytes = bytes;
            }
            HIP_TRY(ws.frame_meta.ensure(bytes));
            h = ws.host_meta;
            d = static_cast<char *>(ws.frame_meta.p);
        }
        for (int c = 0; c < ncodes; ++c) std::memcpy(h + sizeof(DevCode) * c, &codes[c]->dc, sizeof(DevCode));
        int64_t *h_loff = reinterpret_cast<int64_t *>(h + tbl_bytes);
        int64_t *h_xoff = h_loff + nframes;
        int32_t *h_cof = reinterpret_cast<int32_t *>(h_xoff + nframes);
        for (int f = 0; f < nframes; ++f) {
            h_loff[f] = llr_off ? llr_off[f] : (int64_t)f * codes[0]->dc.n;
            h_xoff[f] = x_off ? x_off[f] : (int64_t)f * codes[0]->dc.n;
            h_cof[f] = code_of_frame ? code_of_frame[f] : 0;
        }
        if (ordered) {
            int32_t *h_ord = h_cof + nframes;
            for (int f = 0; f < nframes; ++f) h_ord[f] = f;
            std::stable_sort(h_ord, h_ord + nframes, [&](int a, int b) {
                return codes[code_of_frame[a]]->dc.E > codes[code_of_frame[b]]->dc.E;
            });
        }
        HIP_TRY(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, stream));
        codes_dev = reinterpret_cast<const DevCode *>(d);
        fb.llr_off = reinterpret_cast<const int64_t *>(d + tbl_bytes);
        fb.x_off = fb.llr_off + nframes;
        if (code_of_frame) fb.code_of_frame = reinterpret_cast<const int32_t *>(fb.x_off + nframes);
        if (ordered) fb.order = fb.code_of_frame + nframes;
    }
    // invalid-input flags for every frame, read by the decode kernels
    {
        hipError_t e = launch_check_finite(codes_dev, fb, stream);
        if (e != hipSuccess) return fail(LPDEC_EDEVICE, "input check launch failed: %s", hipGetErrorString(e));
    }
    IterParams ip{};
    ip.mu_inv = 1.0f / p.mu;
    ip.rho = p.rho;
    ip.tol2 = p.tol * p.tol;
    ip.max_iter = p.max_iter;
    StateIO sio{};
    if (state_flags & LPDEC_STATE_IN) {
        sio.z_in = z_state;
        sio.u_in = u_state;
    }
    if (state_flags & LPDEC_STATE_OUT) {
        sio.z_out = z_state;
        sio.u_out = u_state;
    }
    StreamArgs sa{};

    if (cfg.form == Form::Resident || cfg.form == Form::PersistentGlobal) {
        cfg.grid = occupancy_grid(cfg, nframes, codes[0]);
        // per-workgroup scratch (bytes per workgroup of each buffer; 0: not used)
        const WgBytes wb = wg_bytes(s, cfg);
        const bool need_gmu = wb.gmu > 0;
        const bool pg = cfg.form == Form::PersistentGlobal;
        const size_t b_gmu = wb.gmu, b_state = wb.state, b_xprev = wb.xprev, b_slots = wb.slots;
        void *p_queue, *p_gmu, *p_state, *p_xprev, *p_slots;
        if (arena) {
            // queue counter, metadata, then each buffer 256-byte aligned; the grid is
            // cut so that all of them fit (a frame's result does not depend on the grid)
            const size_t per_wg = b_gmu + b_state + b_xprev + b_slots, fixed = 256 + meta_bytes + 4 * 255;
            if (per_wg > 0) {
                if (fixed + per_wg > arena->bytes)
                    return fail(LPDEC_EUNSUPPORTED,
                                "one workgroup of this code needs %zu bytes of scratch; the allocation-free decode "
                                "holds %zu",
                                fixed + per_wg, arena->bytes);
                cfg.grid = (int)std::min<size_t>((size_t)cfg.grid, (arena->bytes - fixed) / per_wg);
            }
            auto align = [](size_t b) { return (b + 255) / 256 * 256; };
            size_t off = 0;
            auto carve = [&](size_t per) -> void * {
                void *q = arena->base + off;
                off += align(per * (size_t)cfg.grid);
                return per ? q : nullptr;
            };
            p_queue = arena->base;
            off = 256 + meta_bytes;
            p_gmu = carve(b_gmu);
            p_state = carve(b_state);
            p_xprev = carve(b_xprev);
            p_slots = carve(b_slots);
            if (off > arena->bytes) return fail(LPDEC_EINVAL, "internal: scratch layout exceeds the arena");
        } else {
            HIP_TRY(ws.queue.ensure(sizeof(int)));
            p_queue = ws.queue.p;
            p_gmu = p_state = p_xprev = p_slots = nullptr;
            if (b_gmu) {
                HIP_TRY(ws.gmu.ensure(b_gmu * cfg.grid));
                p_gmu = ws.gmu.p;
            }
            if (b_state) {
                HIP_TRY(ws.gstate.ensure(b_state * cfg.grid));
                p_state = ws.gstate.p;
            }
            if (b_xprev) {
                HIP_TRY(ws.gxprev.ensure(b_xprev * cfg.grid));
                p_xprev = ws.gxprev.p;
            }
            if (b_slots) {
                HIP_TRY(ws.gslots.ensure(b_slots * cfg.grid));
                p_slots = ws.gslots.p;
            }
        }
        fb.queue = static_cast<int *>(p_queue);
        HIP_TRY(launch_fill_i32(fb.queue, 0, 1, stream));  // a kernel, not a memset: safe under graph capture
        if (need_gmu) {
            sa.gmu = static_cast<float *>(p_gmu);
            sa.gmu_stride = s.nmax;
        }
        if (pg) {
            sa.z = p_state;  // z of every workgroup, then u (FP32, or FP16 values)
            sa.u = static_cast<char *>(p_state) + (cfg.half ? 2 : sizeof(float)) * (size_t)cfg.grid * cfg.state_stride;
            if (cfg.slot_mode == 2) {
                sa.gxprev = static_cast<unsigned *>(p_xprev);
                sa.gmu_stride = s.nmax;
            }
            if (cfg.slot_mode == 0) sa.gslots = static_cast<float *>(p_slots);
        }
        hipError_t e = launch_decode(cfg, codes_dev, fb, ip, sio, sa, stream);
        if (e != hipSuccess) return fail(LPDEC_EDEVICE, "decode launch failed: %s", hipGetErrorString(e));
    } else {
        // streamed: state [frames][E_int] in HBM, one launch per iteration
        const size_t esz = half ? 2 : 4;
        const size_t per = (size_t)s.Eint_max;
        HIP_TRY(ws.z.ensure(esz * per * nframes));
        HIP_TRY(ws.u.ensure(esz * per * nframes));
        HIP_TRY(ws.st.ensure(sizeof(StreamFrame) * nframes));
        HIP_TRY(ws.active.ensure(sizeof(int) * 2));
        HIP_TRY(ws.alist.ensure(sizeof(int) * 2 * (size_t)nframes));
        HIP_TRY(ws.alist_cnt.ensure(sizeof(int) * 3));
        if (!ws.host_active) HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&ws.host_active), 2 * sizeof(int)));
        sa.z = ws.z.p;
        sa.u = ws.u.p;
        sa.st = static_cast<StreamFrame *>(ws.st.p);
        sa.active_count = static_cast<int *>(ws.active.p);
        sa.alist = static_cast<int *>(ws.alist.p);
        sa.alist_cnt = static_cast<int *>(ws.alist_cnt.p);
        if (s.permuted) {
            HIP_TRY(ws.gmu.ensure(sizeof(float) * (size_t)nframes * s.nmax));
            sa.gmu = static_cast<float *>(ws.gmu.p);
            sa.gmu_stride = s.nmax;
        }
        cfg.grid = occupancy_grid(cfg, nframes, codes[0]);
        if (cfg.slot_mode == 0) {
            HIP_TRY(ws.gslots.ensure(sizeof(float) * (size_t)cfg.grid * cfg.slot_stride));
            sa.gslots = static_cast<float *>(ws.gslots.p);
        }
        HIP_TRY(launch_stream_init(codes_dev, nframes, cfg, fb, sio, sa, ip, stream));
        // Iterations are issued in blocks; after each block the number of frames
        // still running is copied to pinned memory and checked one block later.
        const int block = 16;
        // Graph replay: a block is one launch of a graph captured once per set of
        // launch arguments (kernel nodes only: the decode and a one-thread kernel that
        // advances the launch index in device memory).  A replay may run launches past
        // max_iter; they find every frame finished and do nothing.
        const bool graph = c0->graph;
        if (graph) {
            HIP_TRY(ws.launch_dev.ensure(sizeof(int)));
            sa.launch_dev = static_cast<int *>(ws.launch_dev.p);
            HIP_TRY(launch_fill_i32(static_cast<int *>(ws.launch_dev.p), 0, 1, stream));
            struct Key {
                LaunchConfig cfg;
                const DevCode *codes;
                FrameBatch fb;
                IterParams ip;
                StateIO sio;
                StreamArgs sa;
            } key;
            std::memset(&key, 0, sizeof key);
            key.cfg = cfg;
            key.codes = codes_dev;
            key.fb = fb;
            key.ip = ip;
            key.sio = sio;
            key.sa = sa;
            const char *kb = reinterpret_cast<const char *>(&key);
            if (!ws.graph || ws.graph_key.size() != sizeof key ||
                std::memcmp(ws.graph_key.data(), kb, sizeof key) != 0) {
                if (ws.graph) HIP_TRY(hipGraphExecDestroy(ws.graph));
                ws.graph = nullptr;
                if (!ws.capture) HIP_TRY(hipStreamCreateWithFlags(&ws.capture, hipStreamNonBlocking));
                HIP_TRY(hipStreamBeginCapture(ws.capture, hipStreamCaptureModeThreadLocal));
                hipError_t ce = hipSuccess;
                for (int k = 0; k < block && ce == hipSuccess; ++k) {
                    ce = launch_decode(cfg, codes_dev, fb, ip, sio, sa, ws.capture);
                    if (ce == hipSuccess) ce = launch_advance(static_cast<int *>(ws.launch_dev.p), ws.capture);
                }
                hipGraph_t g = nullptr;
                const hipError_t ee = hipStreamEndCapture(ws.capture, &g);
                if (ce != hipSuccess || ee != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return fail(LPDEC_EDEVICE, "capturing the iteration block failed: %s",
                                hipGetErrorString(ce != hipSuccess ? ce : ee));
                }
                const hipError_t ie = hipGraphInstantiate(&ws.graph, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ie != hipSuccess) {
                    ws.graph = nullptr;
                    return fail(LPDEC_EDEVICE, "instantiating the iteration block failed: %s", hipGetErrorString(ie));
                }
                ws.graph_key.assign(kb, kb + sizeof key);
            }
        }
        hipEvent_t ev[2] = {nullptr, nullptr};
        HIP_TRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
        int issued = 0, blk = 0;
        lpdec_status rs = LPDEC_OK;
        while (issued < p.max_iter) {
            const int cnt = graph ? block : std::min(block, p.max_iter - issued);
            if (graph) {
                const hipError_t e = hipGraphLaunch(ws.graph, stream);
                if (e != hipSuccess) {
                    rs = fail(LPDEC_EDEVICE, "graph launch failed: %s", hipGetErrorString(e));
                    break;
                }
            } else {
                for (int k = 0; k < cnt; ++k) {
                    ip.launch = issued + k;
                    hipError_t e = launch_decode(cfg, codes_dev, fb, ip, sio, sa, stream);
                    if (e != hipSuccess) {
                        rs = fail(LPDEC_EDEVICE, "streamed launch failed: %s", hipGetErrorString(e));
                        break;
                    }
                }
            }
            if (rs != LPDEC_OK) break;
            issued += cnt;
            const int slot = blk & 1;
            hipError_t e = hipMemcpyAsync(ws.host_active + slot, sa.active_count + ((issued - 1) & 1), sizeof(int),
                                          hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipEventRecord(ev[slot], stream);
            if (e != hipSuccess) {
                rs = fail(LPDEC_EDEVICE, "progress copy failed: %s", hipGetErrorString(e));
                break;
            }
            if (blk > 0) {
                const int prev = slot ^ 1;
                e = hipEventSynchronize(ev[prev]);
                if (e != hipSuccess) {
                    rs = fail(LPDEC_EDEVICE, "progress wait failed: %s", hipGetErrorString(e));
                    break;
                }
                if (ws.host_active[prev] == 0) break;
            }
            ++blk;
        }
        (void)hipEventSynchronize(ev[0]);
        (void)hipEventSynchronize(ev[1]);
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        if (rs != LPDEC_OK) return rs;
        if (sio.z_out) HIP_TRY(launch_stream_export(codes_dev, nframes, s.Eint_max, half, sio, sa, stream));
    }
    return LPDEC_OK;
}

lpdec_status lpdec_scratch_need(const lpdec_code *code, const lpdec_params *pin, int nframes, bool scattered,
                                ScratchNeed *out) {
    lpdec_params p = pin ? *pin : lpdec_default_params();
    lpdec_status st = check_params(&p);
    if (st != LPDEC_OK) return st;
    const Shape s = shape_of(&code, 1);
    LaunchConfig cfg{};
    st = resolve_config(s, p, scattered, &cfg, code);
    if (st != LPDEC_OK) return st;
    *out = ScratchNeed{};
    if (cfg.form == Form::Streamed) {
        out->streamed = true;
        return LPDEC_OK;
    }
    // the grid of a launch of nframes frames (two frames per workgroup only pair
    // when every CU gets two, as in lpdec_decode_core)
    if (cfg.pair && code->tune_variant[static_cast<int>(Form::Resident)] < 1) {
        const DeviceInfo di = device_info();
        if (nframes < 2 * (di.cus > 0 ? di.cus : 256)) resident_config(s, &cfg, 0);
    }
    cfg.grid = occupancy_grid(cfg, std::max(1, nframes), code);
    out->per_wg = wg_bytes(s, cfg).total();
    out->host = scattered ? meta_host_bytes(nframes) : 0;
    out->fixed = 256 + (out->host + 255) / 256 * 256 + 4 * 255;
    out->grid = cfg.grid;
    return LPDEC_OK;
}

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

lpdec_params lpdec_default_params(void) {
    lpdec_params p;
    p.mu = 3.0f;
    p.rho = 1.9f;
    p.max_iter = 1000;
    p.tol = 1e-5f;
    p.storage = LPDEC_STORAGE_FP32;
    p.mode = LPDEC_MODE_AUTO;
    return p;
}

const char *lpdec_last_error(void) { return g_last_error.c_str(); }

lpdec_status lpdec_code_create(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                               lpdec_code **out) {
    if (!out) return fail(LPDEC_EINVAL, "out must not be NULL");
    *out = nullptr;
    std::unique_ptr<lpdec_code> code(new (std::nothrow) lpdec_code());
    if (!code) return fail(LPDEC_ENOMEM, "host allocation failed");
    lpdec_status st = build_plan(m, n, nnz, row_ptr, col_idx, code.get());
    if (st != LPDEC_OK) return st;
    const lpdec_code *one = code.get();
    code->resident_ok = resident_config(shape_of(&one, 1), &code->resident_cfg);
    *out = code.release();
    return LPDEC_OK;
}

void lpdec_code_destroy(lpdec_code *code) {
    if (!code) return;
    {
        std::lock_guard<std::mutex> lk(code->ws.mu);
        if (code->ws.last) (void)hipEventSynchronize(code->ws.last);
    }
    delete code;
}

lpdec_status lpdec_code_get_info(const lpdec_code *code, lpdec_code_info *info) {
    if (!code || !info) return fail(LPDEC_EINVAL, "code and info must not be NULL");
    info->m = code->dc.m;
    info->n = code->dc.n;
    info->nnz = code->dc.E;
    info->min_check_degree = code->dc.dmin;
    info->max_check_degree = code->dc.dmax;
    info->resident_capable = code->resident_ok ? 1 : 0;
    info->threads_per_frame = code->dc.waves * kWave;
    return LPDEC_OK;
}

static int form_of_mode(int32_t mode) {
    switch (mode) {
        case LPDEC_MODE_RESIDENT: return static_cast<int>(Form::Resident);
        case LPDEC_MODE_PERSISTENT_GLOBAL: return static_cast<int>(Form::PersistentGlobal);
        case LPDEC_MODE_STREAMED: return static_cast<int>(Form::Streamed);
        default: return -1;
    }
}

static int32_t mode_of_form(Form f) {
    switch (f) {
        case Form::Resident: return LPDEC_MODE_RESIDENT;
        case Form::PersistentGlobal: return LPDEC_MODE_PERSISTENT_GLOBAL;
        default: return LPDEC_MODE_STREAMED;
    }
}

lpdec_status lpdec_code_launch_info(const lpdec_code *code, const lpdec_params *pin, lpdec_launch_info *out) {
    if (!code || !out) return fail(LPDEC_EINVAL, "code and out must not be NULL");
    lpdec_params p = pin ? *pin : lpdec_default_params();
    lpdec_status st = check_params(&p);
    if (st != LPDEC_OK) return st;
    LaunchConfig cfg{};
    st = resolve_config(shape_of(&code, 1), p, false, &cfg, code);
    if (st != LPDEC_OK) return st;
    KernelQuery q{};
    hipError_t e = decode_query(cfg, &q);
    if (e != hipSuccess) return fail(LPDEC_EDEVICE, "kernel query failed: %s", hipGetErrorString(e));
    out->mode = mode_of_form(cfg.form);
    out->threads = cfg.threads;
    out->lds_bytes = (int32_t)cfg.lds_bytes;
    out->vgprs = q.vgprs;
    out->runtime_blocks_per_cu = q.occupancy;
    out->resource_blocks_per_cu = resource_blocks_per_cu(cfg, q);
    out->blocks_per_cu = blocks_per_cu(cfg, code);
    int nacc = 0;
    if (cfg.form != Form::Resident && cfg.slot_mode == 2)
        acc_held_chunks(shape_of(&code, 1), cfg.form == Form::PersistentGlobal, 0, &nacc, cfg.half);
    if (nacc > 0) {  // index of the held-chunk count among the code's candidates
        const Shape s = shape_of(&code, 1);
        out->variant = 0;
        for (int v = 0; v < nacc; ++v)
            if (acc_held_chunks(s, cfg.form == Form::PersistentGlobal, v, nullptr, cfg.half) == cfg.acc_kr)
                out->variant = v;
    } else if (cfg.form == Form::Streamed) out->variant = cfg.cpt_tmpl == 0 ? 0 : (cfg.staged ? 2 : 1);
    else if (cfg.form == Form::Resident && cfg.dclass == 0 && cfg.dv == 3 && cfg.cpt_tmpl == 2)
        out->variant = cfg.pair ? 1 : 0;
    else out->variant = -1;
    return LPDEC_OK;
}

lpdec_status lpdec_code_set_tuning(lpdec_code *code, int32_t mode, int32_t bpc, int32_t variant) {
    if (!code) return fail(LPDEC_EINVAL, "code must not be NULL");
    const int f = form_of_mode(mode);
    if (f < 0) return fail(LPDEC_EINVAL, "mode must be RESIDENT, STREAMED or PERSISTENT_GLOBAL (got %d)", mode);
    if (bpc < 0 || bpc > 32) return fail(LPDEC_EINVAL, "blocks_per_cu must lie in 0..32 (got %d)", bpc);
    if (variant < -1 || variant >= LPDEC_TUNE_VARIANTS)
        return fail(LPDEC_EINVAL, "variant must lie in -1..%d (got %d)", LPDEC_TUNE_VARIANTS - 1, variant);
    code->tune_bpc[f] = bpc;
    code->tune_variant[f] = variant;
    return LPDEC_OK;
}

lpdec_status lpdec_autotune(lpdec_code *code, int32_t batch, const float *llr, const lpdec_params *pin,
                            int32_t max_bpc, int32_t *best_out, float *ms_out, void *stream_v) {
    if (!code || !llr) return fail(LPDEC_EINVAL, "code and llr must not be NULL");
    if (batch < 1) return fail(LPDEC_EINVAL, "batch must be >= 1");
    if (max_bpc < 1 || max_bpc > 32) return fail(LPDEC_EINVAL, "max_blocks_per_cu must lie in 1..32");
    lpdec_params p = pin ? *pin : lpdec_default_params();
    lpdec_status st = check_params(&p);
    if (st != LPDEC_OK) return st;
    LaunchConfig cfg{};
    const lpdec_code *one = code;
    st = resolve_config(shape_of(&one, 1), p, false, &cfg, nullptr);
    if (st != LPDEC_OK) return st;
    const int f = static_cast<int>(cfg.form);
    // resident: one or two frames per workgroup, where the code allows both
    bool res_pair = false;
    if (cfg.form == Form::Resident) {
        LaunchConfig probe{};
        res_pair = resident_config(shape_of(&one, 1), &probe, 1) && probe.pair;
    }
    int nacc = 0;  // held-chunk candidates of the large-code kernel
    if (cfg.form != Form::Resident && cfg.slot_mode == 2)
        acc_held_chunks(shape_of(&one, 1), cfg.form == Form::PersistentGlobal, 0, &nacc, cfg.half);
    const int nvar = std::min(LPDEC_TUNE_VARIANTS, nacc > 0 ? nacc : (cfg.form == Form::Streamed ? 3 : (res_pair ? 2 : 1)));
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    const size_t n = (size_t)code->dc.n;
    float *x = nullptr;
    int32_t *it = nullptr;
    uint8_t *fl = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int saved = code->tune_bpc[f], saved_var = code->tune_variant[f];
    int best = 0, best_var = -1;
    float best_ms = 0.0f;
    if (ms_out)
        for (int k = 0; k < LPDEC_TUNE_VARIANTS * max_bpc; ++k) ms_out[k] = -1.0f;
    auto run = [&]() -> lpdec_status {
        HIP_TRY(hipMalloc(&x, sizeof(float) * n * batch));
        HIP_TRY(hipMalloc(&it, sizeof(int32_t) * batch));
        HIP_TRY(hipMalloc(&fl, batch));
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        for (int v = 0; v < nvar; ++v) {
            const int var = nvar == 1 ? -1 : v;
            code->tune_variant[f] = var;
            if (cfg.form == Form::Streamed && nacc == 0) {  // a streamed variant the code does not allow falls back: skip it
                LaunchConfig probe{};
                streamed_config(shape_of(&one, 1), p.storage == LPDEC_STORAGE_FP16, &probe, var);
                const int got = probe.cpt_tmpl == 0 ? 0 : (probe.staged ? 2 : 1);
                if (got != var) continue;
            }
            for (int b = 0; b <= max_bpc; ++b) {
                code->tune_bpc[f] = b == 0 ? 1 : b;  // b = 0: untimed warm-up
                HIP_TRY(hipEventRecord(e0, stream));
                lpdec_status r = lpdec_decode_core(&one, 1, batch, nullptr, nullptr, nullptr, llr, &p, x, it, fl,
                                                   nullptr, nullptr, 0, stream, nullptr, nullptr);
                if (r != LPDEC_OK) return r;
                HIP_TRY(hipEventRecord(e1, stream));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (b == 0) continue;
                if (ms_out) ms_out[v * max_bpc + b - 1] = ms;
                if (best == 0 || ms < best_ms) { best = b; best_var = var; best_ms = ms; }
            }
        }
        return LPDEC_OK;
    };
    st = run();
    if (x) (void)hipFree(x);
    if (it) (void)hipFree(it);
    if (fl) (void)hipFree(fl);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != LPDEC_OK) {
        code->tune_bpc[f] = saved;
        code->tune_variant[f] = saved_var;
        return st;
    }
    code->tune_bpc[f] = best;
    code->tune_variant[f] = best_var;
    if (best_out) {
        best_out[0] = best;
        best_out[1] = best_var;
    }
    return LPDEC_OK;
}

lpdec_status lpdec_code_set_graph(lpdec_code *code, int32_t enable) {
    if (!code) return fail(LPDEC_EINVAL, "code must not be NULL");
    if (enable != 0 && enable != 1) return fail(LPDEC_EINVAL, "enable must be 0 or 1 (got %d)", enable);
    code->graph = enable != 0;
    return LPDEC_OK;
}

lpdec_status lpdec_autotune_multi(const lpdec_code *const *codes, int32_t ncodes, int32_t nframes,
                                  const int32_t *code_of_frame, const int64_t *llr_offset, const float *llr,
                                  int64_t llr_len, const lpdec_params *pin, int32_t max_bpc, int32_t *best_out,
                                  float *ms_out, void *stream_v) {
    if (!codes || ncodes < 1 || !code_of_frame || !llr_offset || !llr)
        return fail(LPDEC_EINVAL, "codes, code_of_frame, llr_offset and llr must not be NULL");
    for (int c = 0; c < ncodes; ++c)
        if (!codes[c]) return fail(LPDEC_EINVAL, "codes[%d] is NULL", c);
    if (nframes < 1) return fail(LPDEC_EINVAL, "nframes must be >= 1");
    if (max_bpc < 1 || max_bpc > 32) return fail(LPDEC_EINVAL, "max_blocks_per_cu must lie in 1..32");
    lpdec_params p = pin ? *pin : lpdec_default_params();
    lpdec_status st = check_params(&p);
    if (st != LPDEC_OK) return st;
    if (p.mode != LPDEC_MODE_AUTO || p.storage != LPDEC_STORAGE_FP32)
        return fail(LPDEC_EINVAL, "the multi-code tuner picks the form: pass mode AUTO and FP32 storage");
    for (int f = 0; f < nframes; ++f) {
        const int c = code_of_frame[f];
        if (c < 0 || c >= ncodes) return fail(LPDEC_EINVAL, "frame %d: code index %d out of range", f, c);
        if (llr_offset[f] < 0 || llr_offset[f] + codes[c]->dc.n > llr_len)
            return fail(LPDEC_EINVAL, "frame %d: llr range outside llr_len %lld", f, (long long)llr_len);
    }
    lpdec_code *lead = const_cast<lpdec_code *>(codes[0]);
    const Shape s = shape_of(codes, ncodes);
    LaunchConfig probe{};
    const bool res_ok = resident_config(s, &probe);
    const int forms[2] = {LPDEC_MODE_RESIDENT, LPDEC_MODE_PERSISTENT_GLOBAL};
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    if (ms_out)
        for (int k = 0; k < 4 * max_bpc; ++k) ms_out[k] = -1.0f;
    const int saved_bpc[2] = {lead->tune_bpc[0], lead->tune_bpc[1]}, saved_order = lead->tune_order;
    float *x = nullptr;
    int32_t *it = nullptr;
    uint8_t *fl = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best[3] = {0, 0, -1};
    float best_ms = 0.0f;
    auto run = [&]() -> lpdec_status {
        HIP_TRY(hipMalloc(&x, sizeof(float) * (size_t)llr_len));
        HIP_TRY(hipMalloc(&it, sizeof(int32_t) * nframes));
        HIP_TRY(hipMalloc(&fl, nframes));
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        for (int fi = 0; fi < 2; ++fi) {
            if (forms[fi] == LPDEC_MODE_RESIDENT && !res_ok) continue;
            const int form = form_of_mode(forms[fi]);
            lpdec_params q = p;
            q.mode = forms[fi];
            for (int order = 0; order < 2; ++order) {
                lead->tune_order = order;
                for (int b = 0; b <= max_bpc; ++b) {
                    lead->tune_bpc[form] = b == 0 ? 1 : b;  // b = 0: untimed warm-up
                    HIP_TRY(hipEventRecord(e0, stream));
                    lpdec_status r = lpdec_decode_core(codes, ncodes, nframes, code_of_frame, llr_offset, llr_offset,
                                                       llr, &q, x, it, fl, nullptr, nullptr, 0, stream, nullptr,
                                                       nullptr);
                    if (r != LPDEC_OK) return r;
                    HIP_TRY(hipEventRecord(e1, stream));
                    HIP_TRY(hipEventSynchronize(e1));
                    float ms = 0.0f;
                    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                    if (b == 0) continue;
                    if (ms_out) ms_out[(fi * 2 + order) * max_bpc + b - 1] = ms;
                    if (best[2] < 0 || ms < best_ms) {
                        best[0] = forms[fi];
                        best[1] = b;
                        best[2] = order;
                        best_ms = ms;
                    }
                }
                lead->tune_bpc[form] = saved_bpc[fi];
            }
        }
        return LPDEC_OK;
    };
    st = run();
    if (x) (void)hipFree(x);
    if (it) (void)hipFree(it);
    if (fl) (void)hipFree(fl);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    lead->tune_bpc[0] = saved_bpc[0];
    lead->tune_bpc[1] = saved_bpc[1];
    lead->tune_order = saved_order;
    if (st != LPDEC_OK) return st;
    lead->tune_bpc[form_of_mode(best[0])] = best[1];
    lead->tune_order = best[2];
    if (best_out) {
        best_out[0] = best[0];
        best_out[1] = best[1];
        best_out[2] = best[2];
    }
    return LPDEC_OK;
}

lpdec_status lpdec_decode(const lpdec_code *code, int32_t batch, const float *llr, const lpdec_params *p,
                          float *x_out, int32_t *iters_out, uint8_t *flags_out, void *stream) {
    if (!code) return fail(LPDEC_EINVAL, "code must not be NULL");
    return lpdec_decode_core(&code, 1, batch, nullptr, nullptr, nullptr, llr, p, x_out, iters_out, flags_out,
                             nullptr, nullptr, 0, stream, nullptr, nullptr);
}

lpdec_status lpdec_decode_state(const lpdec_code *code, int32_t batch, const float *llr, const lpdec_params *p,
                                float *x_out, int32_t *iters_out, uint8_t *flags_out, float *z_state,
                                float *u_state, int32_t state_flags, void *stream) {
    if (!code) return fail(LPDEC_EINVAL, "code must not be NULL");
    if (state_flags & ~(LPDEC_STATE_IN | LPDEC_STATE_OUT)) return fail(LPDEC_EINVAL, "unknown state_flags bits");
    return lpdec_decode_core(&code, 1, batch, nullptr, nullptr, nullptr, llr, p, x_out, iters_out, flags_out,
                             z_state, u_state, state_flags, stream, nullptr, nullptr);
}

lpdec_status lpdec_decode_multi(const lpdec_code *const *codes, int32_t ncodes, int32_t nframes,
                                const int32_t *code_of_frame, const int64_t *llr_offset, const float *llr,
                                int64_t llr_len, const lpdec_params *p, float *x_out, const int64_t *x_offset,
                                int64_t x_len, int32_t *iters_out, uint8_t *flags_out, void *stream) {
    if (!codes || ncodes < 1) return fail(LPDEC_EINVAL, "codes must hold >= 1 code");
    for (int c = 0; c < ncodes; ++c)
        if (!codes[c]) return fail(LPDEC_EINVAL, "codes[%d] is NULL", c);
    if (nframes < 0) return fail(LPDEC_EINVAL, "nframes must be >= 0");
    if (nframes == 0) return LPDEC_OK;
    if (!code_of_frame || !llr_offset || !x_offset)
        return fail(LPDEC_EINVAL, "code_of_frame, llr_offset and x_offset must not be NULL");
    for (int f = 0; f < nframes; ++f) {
        const int c = code_of_frame[f];
        if (c < 0 || c >= ncodes) return fail(LPDEC_EINVAL, "frame %d: code index %d out of range", f, c);
        const int64_t n = codes[c]->dc.n;
        if (llr_offset[f] < 0 || llr_offset[f] + n > llr_len)
            return fail(LPDEC_EINVAL, "frame %d: llr range [%lld, %lld) outside llr_len %lld", f,
                        (long long)llr_offset[f], (long long)(llr_offset[f] + n), (long long)llr_len);
        if (x_offset[f] < 0 || x_offset[f] + n > x_len)
            return fail(LPDEC_EINVAL, "frame %d: x range outside x_len %lld", f, (long long)x_len);
    }
    lpdec_params pp = p ? *p : lpdec_default_params();
    if (pp.mode == LPDEC_MODE_STREAMED || pp.storage == LPDEC_STORAGE_FP16)
        return fail(LPDEC_EUNSUPPORTED, "multi-code decoding runs in one persistent launch (FP32)");
    return lpdec_decode_core(codes, ncodes, nframes, code_of_frame, llr_offset, x_offset, llr, &pp, x_out,
                             iters_out, flags_out, nullptr, nullptr, 0, stream, nullptr, nullptr);
}

lpdec_status lpdec_project(int32_t d, int32_t count, const float *v, float *z, void *stream) {
    if (d < 2 || d > LPDEC_MAX_CHECK_DEGREE)
        return fail(LPDEC_EINVAL, "degree %d outside [2, %d]", d, LPDEC_MAX_CHECK_DEGREE);
    if (count < 0) return fail(LPDEC_EINVAL, "count must be >= 0");
    if (count == 0) return LPDEC_OK;
    if (!v || !z) return fail(LPDEC_EINVAL, "v and z must not be NULL");
    if (v == z) return fail(LPDEC_EINVAL, "z must not alias v");
    hipError_t e = launch_project(d, count, v, z, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(LPDEC_EDEVICE, "projection launch failed: %s", hipGetErrorString(e));
    return LPDEC_OK;
}

}  // extern "C"
