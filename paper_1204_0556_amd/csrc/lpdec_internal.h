// Internal structures shared by the host runtime (lpdec_host.cpp) and the HIP
// kernels (lpdec_kernels.hip) of the same library.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpdec {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxThreads = 1024;  // workgroup limit
constexpr int kMaxWaves = kMaxThreads / kWave;
// LDS staging of the streamed form: one frame's z, u (edges) and gamma/mu (variables)
constexpr int kStageEdges = 8192;
constexpr int kStageVars = 4096;
constexpr int kMaxD = 16;          // LPDEC_MAX_CHECK_DEGREE
constexpr int kAccAllHeld = 8;     // k_decode_acc: held chunks per wave that compile the chunk walk out

// A pointer read from memory (a code table, an argument structure) is generic to
// the compiler, and a generic load also waits on LDS traffic; these mark one as
// pointing to global memory.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *as_global(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *as_global_rw(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// Device view of one code (all pointers are device memory owned by the code).
//
// Checks are grouped by degree and cut into "chunks" of up to 64 checks of one
// degree; one wavefront lane owns one check of a chunk.  A chunk's edge state is
// stored lane-minor: edge k of lane l sits at chunk_off + k*64 + l, so a wave
// touching edge k of its 64 checks reads 256 contiguous bytes.
//
// Variables are renumbered in order of decreasing degree; variable i's edges
// occupy a contiguous "slot" range (its CSC block), in ascending CSR edge order.
// Each edge knows its internal variable and slot.
struct DevCode {
    int m, n, E;          // checks, variables, nnz
    int E_int;            // length of the lane-minor edge arrays (with padding)
    int nchunks;          // chunks of <= 64 checks
    int waves;            // wavefronts per workgroup for this code
    int cpt;              // chunks per wave (chunk c belongs to wave c % waves)
    int dmin, dmax;
    int var_identity;     // internal variable order equals the original one
    int dv;               // common variable degree (0 if degrees differ)
    float dv_inv;         // 1 / dv
    // Variables sorted by decreasing degree form nvc <= 8 classes: class c holds
    // internal variables [vc_start[c], vc_start[c+1]) of degree vc_deg[c], whose
    // slots start at vc_slot0[c].
    int nvc;
    int vc_start[9];
    int vc_slot0[8];
    int vc_deg[8];
    float vc_inv[8];
    const int *chunk_deg;     // [nchunks]
    const int *chunk_off;     // [nchunks] offset into the lane-minor arrays
    const int *chunk_cnt;     // [nchunks] checks in the chunk (<= 64)
    const uint32_t *edge_meta;// [E_int] (slot << 16) | internal variable (0 on padding)
    const uint32_t *edge_acc; // [E_int] 8 x internal variable: byte offset of the edge's
                              // accumulator entry (the accumulator exchange's LDS address)
    const int *edge_csr;      // [E_int] CSR edge id (-1 on padding)
    const int *var_orig;      // [n] internal -> original variable index
    const int2 *var_info;     // [n] {slot0 | deg << 24, bits of 1/deg} per internal variable
};

// Frames of one launch.
struct FrameBatch {
    int nframes;
    const int *code_of_frame;   // device [nframes] or nullptr (all code 0)
    const int64_t *llr_off;     // device [nframes] or nullptr (f * n)
    const float *llr;
    float *x_out;
    const int64_t *x_off;       // device [nframes] or nullptr (f * n)
    int *iters_out;
    uint8_t *flags_out;
    int *queue;                 // device work counter (persistent kernels)
    int *done;                  // optional [nframes] completion flags (host-visible), set last
    const int *order;           // device [nframes] or nullptr: queue position -> frame (persistent forms)
};

struct IterParams {
    float mu_inv;   // 1 / mu
    float rho;
    float tol2;     // tol^2 (threshold = tol^2 * E)
    int max_iter;
    int launch;     // streamed form: iterations already run by every unfinished frame
};

// Optional state input/output in CSR edge order ([frame][E]).
struct StateIO {
    const float *z_in, *u_in;
    float *z_out, *u_out;
};

// Per-frame bookkeeping of the per-iteration (streamed) form.
struct StreamFrame {
    int iter;       // iterations completed
    int done;       // 1 once converged / finished / invalid
};

struct StreamArgs {
    void *z;                // [frames][E_int] fp32 or fp16
    void *u;
    StreamFrame *st;        // [frames]
    int *active_count;      // [2] frames still running after a launch: launch k counts into
                            // entry k & 1 and clears the other one for launch k + 1
    int *alist;             // [2][frames] the frames still running after a launch, in the
                            // order they finished it: launch k appends to half k & 1 and
                            // works through half (k + 1) & 1, dealing its entries to the
                            // workgroups in turn (k_stream_init lists every frame there)
    int *alist_cnt;         // [3] entries of each list: launch k appends at entry k % 3,
                            // reads entry (k + 2) % 3 and clears entry (k + 1) % 3
    float *gslots;          // [workgroups][slot_stride] slot scratch when slots live in global memory
    float *gmu;             // gamma/mu in internal variable order: [workgroups or frames][gmu_stride]
    unsigned *gxprev;       // accumulator mode, persistent form: previous x bits [workgroups][gmu_stride]
    int gmu_stride;
    // streamed form replayed from a captured graph: the launch index lives here
    // (advanced by a one-thread kernel after each launch) instead of in IterParams
    const int *launch_dev;
};

// Launchers (defined in lpdec_kernels.hip).  Return hipSuccess or the launch error.
enum class Form { Resident, PersistentGlobal, Streamed };

struct LaunchConfig {
    Form form;
    int cpt_tmpl;      // register-held chunks per wave: 0 (re-read), 2 or 4
    int vpt_tmpl;      // register-held variables per thread (resident form): 4 or 8
    int dclass;        // 0: degrees exactly 6; 1: degrees 2..8; 2: degrees 6..8 (resident form);
                       // 3: degrees 2..16 (resident form with one chunk per wave, the
                       // persistent-global and streamed forms)
    int dv;            // every variable has this degree (0: mixed), resident form
    int slot_mode;     // 0 global float slots, 1 LDS float slots, 2 LDS fixed-point accumulators
    bool half;         // fp16 state storage (streamed only)
    bool staged;       // streamed: next frame's state staged in LDS by direct-to-LDS loads
    int threads;       // workgroup size
    int grid;          // workgroups
    size_t lds_bytes;  // dynamic LDS
    int lds_E;         // LDS slot array length (x follows it) when slots are in LDS
    int slot_stride;   // per-workgroup stride of global slot scratch (floats)
    int state_stride;  // per-workgroup stride of global state scratch (persistent-global form)
    // resident form, two frames per workgroup (12 waves): for each slot, the virtual
    // wave (the code plan's wave) that physical wave p hosts, in bits 4p..4p+3 (0xF: none)
    bool pair;
    unsigned long long pair_host[2];
    // large check-regular codes with the accumulator exchange: k_decode_acc (acc)
    // with the common check degree and the chunks per wave held in registers
    bool acc;
    int acc_d;
    int acc_kr;
};

hipError_t launch_decode(const LaunchConfig &cfg, const DevCode *codes_dev, const FrameBatch &fb,
                         const IterParams &ip, const StateIO &sio, const StreamArgs &sa,
                         hipStream_t stream);
hipError_t launch_stream_init(const DevCode *codes_dev, int nframes, const LaunchConfig &cfg,
                              const FrameBatch &fb, const StateIO &sio, const StreamArgs &sa,
                              const IterParams &ip, hipStream_t stream);
// Resources of the kernel a configuration selects, and the runtime's occupancy
// estimate for it (workgroups per compute unit).
struct KernelQuery {
    int occupancy;
    int vgprs;
    int static_lds;
};
hipError_t decode_query(const LaunchConfig &cfg, KernelQuery *q);
hipError_t launch_stream_export(const DevCode *codes_dev, int nframes, int E_int, bool half, const StateIO &sio,
                                const StreamArgs &sa, hipStream_t stream);
hipError_t launch_project(int d, int count, const float *v, float *z, hipStream_t stream);
hipError_t launch_fill_i32(int *p, int value, int count, hipStream_t stream);
hipError_t launch_advance(int *p, hipStream_t stream);  // *p += 1 (one thread)

}  // namespace lpdec
