// HIP kernels (gfx950) for ADMM LP decoding.
//
// Paper: Barman, Liu, Draper, Recht, "Decomposition Methods for Large Scale LP
// Decoding" (arXiv 1204.0556).  One iteration of Algorithm 1 (Sec. 3.3), with
// the over-relaxation of Sec. 5.2, is three phases over one frame, executed by
// one workgroup:
//   A  each check lane writes w_e = z_e - u_e (u = lambda/mu) into the slot of
//      edge e; a variable's slots are contiguous (its CSC block)
//   B  x_i = Pi_[0,1]( (sum_slots w - gamma_i/mu) / |N_v(i)| )          (Sec. 3.2)
//   C  per check: v = rho x + (1 - rho) z + u, z' = Pi_PPd(v)  (Sec. 3.2, Alg. 2),
//      u' = v - z', and the two residuals of the stopping rule (Alg. 1)
// Phases are separated by workgroup barriers; slot and x exchanges go through
// LDS (or, for codes too large for LDS, a per-workgroup global scratch).  Sums
// use a fixed order, so a frame's result does not depend on what else runs.
//
// Forms (template flags):
//   RES      the frame's z,u stay in registers across iterations (persistent)
//   PERSIST  one launch decodes frames to completion, pulling frame indices
//            from an atomic queue (per-frame early termination)
//   neither  one launch = one iteration for every unfinished frame; z,u live in
//            HBM between launches (FP32 or FP16 storage)
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lpdec_internal.h"

namespace lpdec {

__device__ __forceinline__ float clamp01(float a) { return __builtin_amdgcn_fmed3f(a, 0.0f, 1.0f); }

// Frames with a non-finite LLR are found before the decode by k_check_finite
// (lpdec_aux.hip, compiled with NaN semantics), which marks them 0x80 in flags_out;
// this file is compiled with -fno-honor-nans and never tests for NaN itself.
__device__ __forceinline__ bool frame_invalid(const FrameBatch &fb, int f) {
    return (__builtin_amdgcn_readfirstlane(fb.flags_out[f]) & 0x80) != 0;
}

// ---------------------------------------------------------------------------
// Check-node operation: Euclidean projection onto PP_d (Sec. 4).
//
// With zhat = Pi_[0,1](v) and r the even floor of ||zhat||_1 (Lemma
// const_parity), the projection is zhat when r = d or f_r^T zhat <= r (f_r =
// +1 on the r+1 largest entries, -1 elsewhere; Alg. 2's early returns), and
// otherwise z(beta) = Pi_[0,1](v - beta f_r) with f_r^T z(beta_opt) = r on
// [0, beta_max] (Lemma optimality).  By the proposition of Sec. 4.4 only the
// breakpoints E1 = {v_k - 1 : k <= r+1} and E2 = {-v_k : k >= r+2} matter, and
// on [0, beta_opt] f_r^T z(beta) equals sum_k min(c_k, a_k - beta) with
// (a_k, c_k) = (v_k, 1) on the top entries and (-v_k, 0) on the others: a
// concave decreasing function, the minimum of the lines
//     L_S(beta) = sum_{k in S} (a_k - beta) + sum_{k not in S} c_k ,  S != {} .
// Its root is therefore the smallest root of those lines,
//     beta_opt = min_S (1 + sum_{k in S} b_k) / |S| ,   b_k = a_k - c_k,
// and for a given |S| = p the best S is the p smallest breakpoints.  In sorted
// order the breakpoints s_k - 1 (k <= r) then -s_k (k > r) form a V-shaped
// (bitonic) list, so one bitonic merge sorts them; beta_opt is then the least
// prefix average.  Everything is branch-free after the early returns and uses
// only static register indices.
// ---------------------------------------------------------------------------
#define LPD_CE(a, b)                                   \
    {                                                  \
        const float _p = s[a], _q = s[b];              \
        s[a] = fmaxf(_p, _q);                          \
        s[b] = fminf(_p, _q);                          \
    }
#include "sortnet.inc"

template <int D>
__device__ __forceinline__ void sort_desc(float *s) {
    if constexpr (D == 2) { LPD_NET_2 }
    else if constexpr (D == 3) { LPD_NET_3 }
    else if constexpr (D == 4) { LPD_NET_4 }
    else if constexpr (D == 5) { LPD_NET_5 }
    else if constexpr (D == 6) { LPD_NET_6 }
    else if constexpr (D == 7) { LPD_NET_7 }
    else if constexpr (D == 8) { LPD_NET_8 }
    else if constexpr (D == 9) { LPD_NET_9 }
    else if constexpr (D == 10) { LPD_NET_10 }
    else if constexpr (D == 11) { LPD_NET_11 }
    else if constexpr (D == 12) { LPD_NET_12 }
    else if constexpr (D == 13) { LPD_NET_13 }
    else if constexpr (D == 14) { LPD_NET_14 }
    else if constexpr (D == 15) { LPD_NET_15 }
    else if constexpr (D == 16) { LPD_NET_16 }
}
#undef LPD_CE

template <int P>
__device__ __forceinline__ void bitonic_merge_asc(float *b) {
#pragma unroll
    for (int k = P / 2; k >= 1; k >>= 1) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
            if ((i & k) == 0) {
                const float p = b[i], q = b[i + k];
                b[i] = fminf(p, q);
                b[i + k] = fmaxf(p, q);
            }
        }
    }
}

template <int D>
__device__ __forceinline__ void project_pp(const float *v, float *z) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        z[k] = clamp01(v[k]);
        s += z[k];
    }
    const float rf = 2.0f * floorf(0.5f * s);  // constituent parity r
    if (rf >= (float)D) return;                 // r = d
    float sv[D];
#pragma unroll
    for (int k = 0; k < D; ++k) sv[k] = v[k];
    sort_desc<D>(sv);
    // f_r^T zhat = 2 (sum of the r+1 largest clipped entries) - sum of all of them
    float top = clamp01(sv[0]);
    {
        float pref = top;
#pragma unroll
        for (int k = 1; k < D; ++k) {
            pref += clamp01(sv[k]);
            if ((k & 1) == 0) top = (rf == (float)k) ? pref : top;
        }
    }
    const float g0 = 2.0f * top - s;
    if (g0 <= rf) return;  // zhat lies in PP_d
    // t1 = v_(r+1), t2 = v_(r+2) (1-based order statistics); r is even
    float t1 = sv[0];
    float t2 = (D > 1) ? sv[1] : -INFINITY;
#pragma unroll
    for (int k = 2; k < D; k += 2) {
        if (rf == (float)k) {
            t1 = sv[k];
            t2 = (k + 1 < D) ? sv[k + 1] : -INFINITY;
        }
    }
    const bool all_top = (rf + 1.0f >= (float)D);
    if (!all_top && !(t1 > t2)) return;  // beta_max = 0
    const float beta_max = all_top ? t1 : 0.5f * (t1 - t2);
    constexpr int P = (D <= 2) ? 2 : ((D <= 4) ? 4 : ((D <= 8) ? 8 : 16));
    float bp[P];
#pragma unroll
    for (int k = 0; k < P; ++k)
        bp[k] = (k < D) ? (((float)k <= rf) ? sv[k] - 1.0f : -sv[k]) : INFINITY;
    bitonic_merge_asc<P>(bp);
    float acc = 1.0f, beta = INFINITY;
#pragma unroll
    for (int p = 1; p <= D; ++p) {
        acc += bp[p - 1];
        beta = fminf(beta, acc * (1.0f / (float)p));
    }
    beta = fminf(fmaxf(beta, 0.0f), beta_max);
#pragma unroll
    for (int k = 0; k < D; ++k) z[k] = clamp01(fmaf((v[k] >= t1) ? -1.0f : 1.0f, beta, v[k]));
}

// ---------------------------------------------------------------------------
// Standalone check-node kernel (lpdec_project): one lane per vector.
template <int D>
__global__ void __launch_bounds__(256) k_project(int count, const float *__restrict__ v,
                                                 float *__restrict__ z) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    float a[D], b[D];
#pragma unroll
    for (int k = 0; k < D; ++k) a[k] = v[(size_t)t * D + k];
    project_pp<D>(a, b);
#pragma unroll
    for (int k = 0; k < D; ++k) z[(size_t)t * D + k] = b[k];
}

hipError_t launch_project(int d, int count, const float *v, float *z, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const dim3 block(256), grid((count + 255) / 256);
    switch (d) {
        case 2: hipLaunchKernelGGL(k_project<2>, grid, block, 0, stream, count, v, z); break;
        case 3: hipLaunchKernelGGL(k_project<3>, grid, block, 0, stream, count, v, z); break;
        case 4: hipLaunchKernelGGL(k_project<4>, grid, block, 0, stream, count, v, z); break;
        case 5: hipLaunchKernelGGL(k_project<5>, grid, block, 0, stream, count, v, z); break;
        case 6: hipLaunchKernelGGL(k_project<6>, grid, block, 0, stream, count, v, z); break;
        case 7: hipLaunchKernelGGL(k_project<7>, grid, block, 0, stream, count, v, z); break;
        case 8: hipLaunchKernelGGL(k_project<8>, grid, block, 0, stream, count, v, z); break;
        case 9: hipLaunchKernelGGL(k_project<9>, grid, block, 0, stream, count, v, z); break;
        case 10: hipLaunchKernelGGL(k_project<10>, grid, block, 0, stream, count, v, z); break;
        case 11: hipLaunchKernelGGL(k_project<11>, grid, block, 0, stream, count, v, z); break;
        case 12: hipLaunchKernelGGL(k_project<12>, grid, block, 0, stream, count, v, z); break;
        case 13: hipLaunchKernelGGL(k_project<13>, grid, block, 0, stream, count, v, z); break;
        case 14: hipLaunchKernelGGL(k_project<14>, grid, block, 0, stream, count, v, z); break;
        case 15: hipLaunchKernelGGL(k_project<15>, grid, block, 0, stream, count, v, z); break;
        case 16: hipLaunchKernelGGL(k_project<16>, grid, block, 0, stream, count, v, z); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ void k_fill_i32(int *p, int value, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = value;
}

hipError_t launch_fill_i32(int *p, int value, int count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((count + 255) / 256), dim3(256), 0, stream, p, value, count);
    return hipGetLastError();
}

__global__ void k_advance(int *p) {
    if (threadIdx.x == 0) *p += 1;
}

hipError_t launch_advance(int *p, hipStream_t stream) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, stream, p);
    return hipGetLastError();
}

// A value every lane of the wave holds (a frame's code index or offsets), moved to
// scalar registers so that what is addressed through it (the frame's code table,
// its LLR and x rows) is addressed with scalar arithmetic.
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Streamed form: iterations every unfinished frame has run before this launch --
// from the launch's arguments, or from device memory when the launches are
// replayed from a captured graph (whose arguments are fixed).
__device__ __forceinline__ int streamed_launch(const IterParams &ip, const StreamArgs &sa) {
    return sa.launch_dev ? __builtin_amdgcn_readfirstlane(*as_global(sa.launch_dev)) : ip.launch;
}

// ---------------------------------------------------------------------------
// Workgroup helpers.

// Sum over the 64 lanes of a wavefront, returned in every lane.  DPP steps sum
// each row of 16 lanes (quad_perm xor 1, xor 2, half-row mirror, row mirror; every
// lane of a row ends with bitwise the same value since float addition commutes).
// Two row broadcasts then combine the row sums R0..R3: lane 15 of rows 0 and 2 into
// rows 1 and 3 (R1 + R0, R3 + R2), lane 31 into row 3 ((R3 + R2) + (R1 + R0)), read
// from lane 63 -- by commutativity bitwise (R0 + R1) + (R2 + R3).  No LDS traffic,
// and the same order in every wave and every kernel form.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_shift(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xF, ROWS == 0xF));
}
__device__ __forceinline__ float wave_sum(float x) {
    x += dpp_shift<0xB1>(x);         // quad_perm [1,0,3,2]
    x += dpp_shift<0x4E>(x);         // quad_perm [2,3,0,1]
    x += dpp_shift<0x141>(x);        // row_half_mirror
    x += dpp_shift<0x140>(x);        // row_mirror
    x += dpp_shift<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3 (rows 0, 2 add 0)
    x += dpp_shift<0x143, 0x8>(x);   // row_bcast:31 into row 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}
// wave_sum of values that are +0 outside lanes 0..15 and never -0 (the per-wave
// residual partials of the stopping test, one lane per wave of the workgroup): the
// other rows sum to +0, and R0 + (+0) = R0, so the row steps alone give the same bits.
__device__ __forceinline__ float row0_sum(float x) {
    x += dpp_shift<0xB1>(x);
    x += dpp_shift<0x4E>(x);
    x += dpp_shift<0x141>(x);
    x += dpp_shift<0x140>(x);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
}

// Workgroup barrier.  With LDS_ONLY the release/acquire fences cover LDS only, so
// global stores still in flight (the previous phase's z, u) do not have to land
// first; the phases exchange data through LDS alone in every form but the
// global-slot one.
template <bool LDS_ONLY>
__device__ __forceinline__ void wg_barrier() {
    if constexpr (LDS_ONLY) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    } else {
        __syncthreads();
    }
}

// Barrier for the LDS-staged streamed form: this wave's LDS operations complete,
// then s_barrier.  Unlike a fenced barrier it does not wait for the direct-to-LDS
// loads of the next frame's state, which stay in flight across the phases; the
// "memory" clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier_nofence() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}
// Wait for this wave's outstanding vector-memory operations.  A real s_waitcnt
// (vmcnt 0; expcnt and lgkmcnt left at their maxima) rather than inline asm, so
// the compiler's wait-count tracking knows that every earlier load has landed.
__device__ __forceinline__ void vmem_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// Direct-to-LDS loads: lane l's 16 (4) bytes from src land at lds_base + 16 l (4 l);
// lds_base must be the same in every lane of the wave.  (Kept out of lambdas: a
// target builtin inside a lambda of a kernel template suppresses the kernel's
// host-side launch stub.)
__device__ __forceinline__ void lds_copy16(const float *src, float *lds_base) {
    __builtin_amdgcn_global_load_lds(src, lds_base, 16, 0, 0);
}
__device__ __forceinline__ void lds_copy4(const float *src, float *lds_base) {
    __builtin_amdgcn_global_load_lds(src, lds_base, 4, 0, 0);
}


// The same pointer, hidden from the optimiser (loads through it are not moved
// out of the loop they are written in).
template <typename T>
__device__ __forceinline__ const T *opaque_ptr(const T *p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Row `off` (wave-uniform) of a lane-minor table, its address in scalar registers.
__device__ __forceinline__ const __attribute__((address_space(1))) int *csr_row(const int *table, int off) {
    return as_global(opaque_ptr(table)) + __builtin_amdgcn_readfirstlane(off);
}

// Degree, offset and check count of chunk c (c wave-uniform).
struct ChunkDesc {
    int deg, off, cnt;
};
__device__ __forceinline__ ChunkDesc chunk_desc(const DevCode &C, int c) {
    ChunkDesc h;
    h.deg = __builtin_amdgcn_readfirstlane(as_global(C.chunk_deg)[c]);
    h.off = __builtin_amdgcn_readfirstlane(as_global(C.chunk_off)[c]);
    h.cnt = __builtin_amdgcn_readfirstlane(as_global(C.chunk_cnt)[c]);
    return h;
}

// Packed metadata of one chunk of degree d (0: no chunk) into m[0..D): loads for
// every e, the index clamped to the chunk's last row, so they can be issued
// without branches ahead of their use (rows e >= d repeat row d-1 and are unused).
template <int D>
__device__ __forceinline__ void load_meta(uint32_t *m, const uint32_t *edge_meta, int off, int d, int lane) {
    const int last = max(d, 1) - 1;  // off and d are wave-uniform: each row address is scalar
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const auto row = as_global(edge_meta) + __builtin_amdgcn_readfirstlane(off + min(e, last) * kWave);
        m[e] = row[lane];
    }
}

template <int DMIN, int DMAX, typename F>
__device__ __forceinline__ void dispatch_degree(int d, F &&f) {
    if constexpr (DMIN == DMAX) {
        f(std::integral_constant<int, DMIN>{});
    } else {
        if (d == DMIN) f(std::integral_constant<int, DMIN>{});
        else dispatch_degree<DMIN + 1, DMAX>(d, f);
    }
}

// x-update of one variable from its slots (Sec. 3.2).  Variables are numbered
// by decreasing degree, so the code describes them by at most 8 degree classes.
struct VarLoc {
    int slot0, deg;
    float inv;
};

__device__ __forceinline__ VarLoc var_loc(const DevCode &C, int i) {
    int c = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k)
        if (k < C.nvc && i >= C.vc_start[k]) c = k;
    VarLoc L;
    L.deg = C.vc_deg[c];
    L.slot0 = C.vc_slot0[c] + (i - C.vc_start[c]) * L.deg;
    L.inv = C.vc_inv[c];
    return L;
}

__device__ __forceinline__ float x_update(const float *slots, const VarLoc &L, float gmu) {
    float s = 0.0f;
    for (int p = 0; p < L.deg; ++p) s += slots[L.slot0 + p];
    return clamp01((s - gmu) * L.inv);
}

// Exact, order-independent per-variable sums for codes whose slot array does not
// fit in LDS: each replica difference w (first clamped to [-2^31, 2^31 - 128], the
// largest float below 2^31) is converted to a signed 32.32 fixed-point value and
// accumulated with 64-bit integer LDS atomics.  Integer addition is associative, so
// the sum does not depend on the order the lanes arrive in.  The conversion rounds
// down to a multiple of 2^-32, strictly so for negative w: with t = trunc(|w| 2^32),
// the value is t when the sign bit of w is clear and the bitwise complement of t,
// -t - 1, when it is set (-0.0 included): an error of at most 2^-32 either way.  It is branch-free FP32/integer arithmetic: the
// magnitude splits exactly into its integer part and its fraction (the difference
// of a float and its floor is exact), and the fraction scaled by 2^32 is an exact
// float whose integer part is the low word.
__device__ __forceinline__ unsigned long long to_fixed(float w) {
    const float c = __builtin_amdgcn_fmed3f(w, -2147483648.0f, 2147483520.0f);
    const float a = fabsf(c);
    const float ah = floorf(a);
    const float r = (a - ah) * 4294967296.0f;  // in [0, 2^32)
    const unsigned hi = (unsigned)ah, lo = (unsigned)r;
    const unsigned m = (unsigned)(__float_as_int(c) >> 31);  // all ones when negative
    return ((unsigned long long)(hi ^ m) << 32) | (lo ^ m);
}
// The sum back to FP32: a correctly rounded conversion of the signed 64-bit value
// (integer normalisation, no FP64), then an exact scale by 2^-32.
__device__ __forceinline__ float from_fixed(unsigned long long a) {
    return (float)(long long)a * 0x1p-32f;
}

// The accumulator entry at byte offset off (edge_acc) of the accumulator array.
__device__ __forceinline__ unsigned long long *acc_entry(unsigned long long *acc, uint32_t off) {
    return reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(acc) + off);
}
// LDS byte address a as a pointer.  For a kernel without static LDS the dynamic
// array starts at address 0, so an entry's byte offset is its address: the access
// needs no add of the array's address (a link-time symbol that the compiler does
// not fold into the instruction's offset field).
template <typename T>
__device__ __forceinline__ T *lds_at(uint32_t a) {
    return (T *)(__attribute__((address_space(3))) T *)(size_t)a;
}
// k_decode_acc's residual slots, frame index and certificate votes follow its 8 n
// bytes of accumulators (from the next 16-byte boundary); kAccTailBytes of dynamic LDS
// hold them, the 8 bytes the alignment may skip included.
__host__ __device__ constexpr uint32_t acc_tail_offset(int n) { return (8u * (uint32_t)n + 15u) & ~15u; }
constexpr size_t kAccFrameOffset = sizeof(float) * 2 * 2 * kMaxWaves;  // after s_red
constexpr size_t kAccVoteOffset = kAccFrameOffset + 16;                // two votes per wave
constexpr size_t kAccTailBytes = kAccVoteOffset + sizeof(int) * 2 * kMaxWaves + 16;

// Accumulator exchange, variable phase: x_i of variables tid, tid + NT, ... from
// the variable's accumulator entry (less the previous x its high word still holds,
// kept in xprev by the persistent forms; without xprev the high word is zero),
// written back to the entry's high word and to xprev.  VBA variables per pass: their
// global loads (previous x, gamma/mu, 1/degree) are issued together before the first
// is used, so a pass waits once instead of once per variable.  PREV: xprev is given.
template <int VBA, bool PREV>
__device__ __forceinline__ void acc_x_update(unsigned long long *acc, unsigned *xprev, const float *gsrc,
                                             float gscale, const DevCode &C, int tid, int NT) {
    const auto vinv = as_global(reinterpret_cast<const int *>(C.var_info));
    for (int i0 = tid; i0 < C.n; i0 += VBA * NT) {
        unsigned prev[VBA];
        float g[VBA], inv[VBA];
#pragma unroll
        for (int t = 0; t < VBA; ++t) {
            const int i = i0 + t * NT;
            const bool ok = i < C.n;
            prev[t] = (PREV && ok) ? as_global(xprev)[i] : 0u;
            g[t] = ok ? as_global(gsrc)[i] : 0.0f;
            inv[t] = (C.dv > 0) ? C.dv_inv : (ok ? __int_as_float(vinv[2 * i + 1]) : 0.0f);
        }
#pragma unroll
        for (int t = 0; t < VBA; ++t) {
            const int i = i0 + t * NT;
            if (i < C.n) {
                const unsigned long long a = acc[i] - ((unsigned long long)prev[t] << 32);
                const float x = clamp01((from_fixed(a) - g[t] * gscale) * inv[t]);
                acc[i] = (unsigned long long)__float_as_uint(x) << 32;
                if constexpr (PREV) as_global_rw(xprev)[i] = __float_as_uint(x);
            }
        }
    }
}

// one check update of degree D on registers z,u (length DMAX arrays); x is read
// from xs with stride XS (2 when x shares an accumulator entry)
// (AB: meta holds the accumulator entries' byte offsets, from edge_acc; x then sits
// at that offset from the accumulator array, i.e. at xs + offset - 4 bytes)
template <int D, int XS = 1, bool AB = false>
__device__ __forceinline__ void check_update(float *z, float *u, const uint32_t *meta, const float *xs,
                                             float rho, float &rp, float &rd) {
    float v[D], zn[D], xv[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        xv[k] = AB ? *reinterpret_cast<const float *>(reinterpret_cast<const char *>(xs) + meta[k])
                   : xs[XS * (meta[k] & 0xffffu)];
        v[k] = fmaf(rho, xv[k] - z[k], z[k]) + u[k];  // q + u with q = rho x + (1-rho) z
    }
    project_pp<D>(v, zn);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float dx = xv[k] - zn[k];
        const float dz = zn[k] - z[k];
        rp = fmaf(dx, dx, rp);
        rd = fmaf(dz, dz, rd);
        u[k] = v[k] - zn[k];
        z[k] = zn[k];
    }
}

template <bool HALF>
__device__ __forceinline__ float ld_state(const void *p, size_t i) {
    if constexpr (HALF) return __half2float(__ushort_as_half(as_global(static_cast<const unsigned short *>(p))[i]));
    else return as_global(static_cast<const float *>(p))[i];
}
template <bool HALF>
__device__ __forceinline__ void st_state(void *p, size_t i, float a) {
    if constexpr (HALF) as_global_rw(static_cast<unsigned short *>(p))[i] = __half_as_ushort(__float2half_rn(a));
    else as_global_rw(static_cast<float *>(p))[i] = a;
}
// Two FP16 state values in one register (a in the low half), rounded as st_state rounds
// (to nearest even): one packed conversion instead of two conversions and an OR.
typedef float lpd_f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 lpd_f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_h2(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector((lpd_f32x2){a, b}, lpd_f16x2));
}
__device__ __forceinline__ float lo_h2f(unsigned v) { return __half2float(__ushort_as_half((unsigned short)(v & 0xffffu))); }
__device__ __forceinline__ float hi_h2f(unsigned v) { return __half2float(__ushort_as_half((unsigned short)(v >> 16))); }
// lo - hi of a packed pair in one mixed-precision FMA: lo * 1 + (-hi) with both
// halves read as FP16 and one FP32 rounding, the value lo_h2f(v) - hi_h2f(v) has
// (the compiler rewrites an FMA by 1 into an add of two widened halves, three
// instructions, so it is written out).
__device__ __forceinline__ float packed_diff(unsigned v) {
    float w;
    asm("v_fma_mix_f32 %0, %1, 1.0, -%1 op_sel:[0,0,1] op_sel_hi:[1,0,1]" : "=v"(w) : "v"(v));
    return w;
}

// ---------------------------------------------------------------------------
// The decoder kernel.
//
// Check side: wave w owns chunks c = w + k*C.waves (k < C.cpt); lane l owns
// check l of each of them.  CPT > 0 keeps those chunks' z,u (and packed edge
// metadata) in registers; CPT == 0 walks the chunks and re-reads state.
// Variable side: thread t owns internal variables t, t + NT, ...
// Streamed form with register-held chunks: either the register budget is capped
// so that two workgroups of <= 768 threads share a CU (6 waves per SIMD) and one
// workgroup's memory waits overlap the other's arithmetic, or (STG) one
// workgroup per CU stages the next frame's z, u and gamma/mu into LDS with
// direct-to-LDS loads issued right after the current frame's state has been
// read, so the loads stream in during the current frame's three phases.
template <int DMIN, int DMAX, int CPT, int VPT, bool RES, bool PERSIST, int SM, bool HALF, int MAXT, int DV,
          bool STG>
__global__ void __launch_bounds__(MAXT, (!PERSIST && CPT > 0 && !STG) ? (MAXT <= 768 ? 6 : 4) : 1)
k_decode(const DevCode *__restrict__ codes, FrameBatch fb, IterParams ip, StateIO sio, StreamArgs sa,
         int lds_E, int slot_stride, int state_stride) {
    // SM: where the slot exchange lives -- 0 global float slots, 1 LDS float slots,
    // 2 LDS fixed-point accumulators (x then sits in each entry's high word)
    static_assert(!RES || (CPT > 0 && PERSIST && SM == 1), "register-resident form needs CPT>0");
    static_assert(SM != 2 || CPT == 0, "accumulator mode walks chunks");
    static_assert(!STG || (!PERSIST && CPT > 0 && SM == 1 && !HALF && DMIN == 6 && DMAX == 6 && VPT == 0),
                  "LDS staging: streamed FP32 degree-6 form with register-held chunks");
    constexpr bool LDS_SLOTS = SM == 1;
    constexpr int XS = (SM == 2) ? 2 : 1;
    extern __shared__ __attribute__((aligned(16))) float lds[];  // 64-bit accumulators need 8-byte alignment
    __shared__ float s_red[2][2][kMaxWaves];
    __shared__ int s_frame;
    // LDS staging of one frame (STG): z and u in the lane-minor edge order, gamma/mu
    // in internal variable order
    constexpr int SE = STG ? kStageEdges : 1;
    constexpr int SN = STG ? kStageVars : 1;
    __shared__ __attribute__((aligned(16))) float stg_z[SE];
    __shared__ __attribute__((aligned(16))) float stg_u[SE];
    __shared__ __attribute__((aligned(16))) float stg_g[SN];
    // STG: slots and x in static LDS as well, so that every LDS array is a distinct
    // object and the compiler can tell the staging area's loads from phase traffic
    __shared__ __attribute__((aligned(16))) float stg_slots[SE];
    __shared__ __attribute__((aligned(16))) float stg_x[SN];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    // the wave index in a scalar register lets the chunk walks use scalar
    // arithmetic; the degree 6..8 resident kernel, short of scalar registers
    // already, keeps it in a vector register
    const int wave = (RES && DMAX > 6) ? (tid >> 6) : __builtin_amdgcn_readfirstlane(tid >> 6);
    const int NT = blockDim.x;
    const int NW = NT >> 6;

    float *slots = STG ? stg_slots : (LDS_SLOTS ? lds : (sa.gslots + (size_t)blockIdx.x * slot_stride));
    float *xs = STG ? stg_x : ((SM == 1) ? (lds + lds_E) : ((SM == 2) ? lds + 1 : lds));
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(lds);
    unsigned *xprev = sa.gxprev ? sa.gxprev + (size_t)blockIdx.x * sa.gmu_stride : nullptr;

    constexpr int NC = CPT > 0 ? CPT : 1;
    float z[NC][DMAX], u[NC][DMAX];
    // Packed edge metadata of the register-held chunks: kept in registers for
    // degree-6 codes with up to two chunks per wave; with checks of degree up to 8,
    // or four chunks per wave, the registers hold only z and u, and the metadata
    // (per code, shared by every frame, so L2-resident) is loaded again each
    // iteration, one chunk ahead.
    constexpr bool MREG = DMAX <= 6 && CPT <= 2;
    // register-resident form: phase C writes each chunk's slots for the next
    // iteration right after updating it (phase A fused into phase C; phase C
    // reads only x, never the slots).  With metadata from memory this halves its
    // loads; with two chunks per wave it measured 3 % faster, with one chunk per
    // wave slower, so that variant keeps the separate pass.
    constexpr bool FUSED_A = RES && (!MREG || CPT >= 2);
    // variables per pass of the mixed-degree variable phase (their table entries
    // and gamma/mu are loaded together before the sums)
    constexpr int VB = 4;
    constexpr int GQ = STG ? 4 : 1;  // STG: gamma/mu of this thread's variables tid + t NT
    float gq[GQ];
    constexpr bool LBAR = SM != 0;  // phase barriers need only order LDS
    uint32_t meta[NC][MREG ? DMAX : 1];
    int cdeg[NC], coff[NC];
    bool cval[NC];
    float vg[VPT > 0 ? VPT : 1];
    // owned variables' slot blocks (resident form; DV > 0: every variable has degree DV)
    int vslot[VPT > 0 ? VPT : 1], vdeg[VPT > 0 ? VPT : 1];
    float vinv[VPT > 0 ? VPT : 1];
    int cur_code = -1;

    // Streamed form: this workgroup owns frames blockIdx.x + k*G (G = gridDim.x).
    // Their done-flags are read 64 at a time (one per lane) and the unfinished
    // ones taken from a ballot mask, identical in every wave.
    const int launch = PERSIST ? 0 : streamed_launch(ip, sa);
    // Streamed form: the frames still running after the previous launch, listed in
    // the order they finished it, are dealt to the workgroups in turn (entry
    // blockIdx.x + k G, G = gridDim.x), so every workgroup gets the same number of
    // frames to within one however few remain.  Each frame that stays unfinished
    // appends itself to this launch's list.
    // The list entries are read 64 at a time (one per lane, with their done flags)
    // and the unfinished frames taken from a ballot mask, identical in every wave.
    int lcnt = 0;
    const int *lprev = nullptr;
    if constexpr (!PERSIST) {
        lcnt = min(uniform_i32(sa.alist_cnt[(launch + 2) % 3]), fb.nframes);
        lprev = sa.alist + (size_t)((launch + 1) & 1) * fb.nframes;
        if (blockIdx.x == 0 && tid == 0) {
            sa.active_count[(launch + 1) & 1] = 0;  // next launch's counter
            sa.alist_cnt[(launch + 1) % 3] = 0;     // next launch's list
        }
    }
    int lbase = (int)blockIdx.x - kWave * (int)gridDim.x;
    int lframe = 0;  // this lane's frame of the current group of entries
    unsigned long long lmask = 0ull;
    auto next_active = [&]() -> int {
        for (;;) {
            if (lmask) {
                const int j = __builtin_ctzll(lmask);
                lmask &= lmask - 1ull;
                return __builtin_amdgcn_readlane(lframe, j);
            }
            lbase += kWave * (int)gridDim.x;
            if (lbase >= lcnt) return fb.nframes;
            const int lj = lbase + lane * (int)gridDim.x;
            const int g = lj < lcnt ? lprev[lj] : -1;
            lframe = g;
            lmask = __ballot(g >= 0 && g < fb.nframes && !sa.st[g].done);
        }
    };
    // a frame that stays unfinished: count it and list it for the next launch
    auto list_unfinished = [&](int g) {
        atomicAdd(sa.active_count + (launch & 1), 1);
        const int pos = atomicAdd(sa.alist_cnt + launch % 3, 1);
        if (pos < fb.nframes) sa.alist[(size_t)(launch & 1) * fb.nframes + pos] = g;
    };
    // STG: start the direct-to-LDS copy of frame g's z, u (16 bytes per lane) and
    // gamma/mu (4 bytes per lane); each wave copies every NW-th 1 KB block
    auto stage_issue = [&](const DevCode &Cg, int g) {
        if constexpr (STG) {
            const float *zs = static_cast<const float *>(sa.z) + (size_t)g * Cg.E_int;
            const float *us = static_cast<const float *>(sa.u) + (size_t)g * Cg.E_int;
            for (int c = wave; c < (Cg.E_int + 255) >> 8; c += NW) {
                const int idx = (c << 8) + (lane << 2);
                if (idx < Cg.E_int) {  // E_int is a multiple of 64: idx + 3 < E_int too
                    lds_copy16(zs + idx, stg_z + (c << 8));
                    lds_copy16(us + idx, stg_u + (c << 8));
                }
            }
            const float *gs = Cg.var_identity ? fb.llr + (int64_t)g * Cg.n : sa.gmu + (size_t)g * sa.gmu_stride;
            for (int c = wave; c < (Cg.n + 63) >> 6; c += NW) {
                const int i = (c << 6) + lane;
                if (i < Cg.n) lds_copy4(gs + i, stg_g + (c << 6));
            }
        }
    };
    int pending = -1;  // STG: the next frame, its copy already issued
    for (;;) {
        int f;
        if constexpr (PERSIST) {
            // the frame index and the workgroup votes below are moved to scalar
            // registers: branches on them are then uniform, so the frame loop
            // keeps one shape for all lanes (lane 0 fetches the next frame)
            if (tid == 0) {
                const int q = atomicAdd(fb.queue, 1);
                s_frame = (fb.order && q < fb.nframes) ? fb.order[q] : q;
            }
            __syncthreads();
            f = __builtin_amdgcn_readfirstlane(s_frame);
            __syncthreads();
        } else if constexpr (STG) {
            if (pending < 0) {
                f = next_active();
                if (f < fb.nframes) stage_issue(codes[0], f);
            } else {
                f = pending;
            }
            pending = -1;
            vmem_wait_all();  // this wave's share of frame f's copy has landed
            lds_barrier_nofence();
        } else {
            f = next_active();
        }
        if (f >= fb.nframes) break;

        const int ci = fb.code_of_frame ? uniform_i32(fb.code_of_frame[f]) : 0;
        const DevCode &C = codes[ci];
        const int64_t loff = fb.llr_off ? uniform_i64(fb.llr_off[f]) : (int64_t)f * C.n;
        const float *gam = fb.llr + loff;
        const float thr = ip.tol2 * (float)C.E;
        float *gmu_row = sa.gmu ? sa.gmu + (size_t)(PERSIST ? blockIdx.x : f) * sa.gmu_stride : nullptr;

        // streamed form: unfinished frames advance in lockstep, one iteration per launch
        const int iter0 = launch;

        // -- per-code register metadata -------------------------------------
        if constexpr (CPT > 0) {
            if (ci != cur_code) {
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    const int c = wave + k * C.waves;
                    const bool has = (wave < C.waves) && (k < C.cpt) && (c < C.nchunks);
                    const ChunkDesc h = has ? chunk_desc(C, c) : ChunkDesc{0, 0, 0};
                    cdeg[k] = h.deg;
                    coff[k] = h.off;
                    cval[k] = lane < h.cnt;
                    if constexpr (MREG) {
#pragma unroll
                        for (int e = 0; e < DMAX; ++e)
                            meta[k][e] = (cval[k] && e < cdeg[k]) ? C.edge_meta[coff[k] + e * kWave + lane] : 0u;
                    }
                }
                if constexpr (VPT > 0 && DV == 0) {
#pragma unroll
                    for (int t = 0; t < VPT; ++t) {
                        const int i = tid + t * NT;
                        VarLoc L{0, 0, 0.0f};
                        if (i < C.n) L = var_loc(C, i);
                        vslot[t] = L.slot0;
                        vdeg[t] = L.deg;
                        vinv[t] = L.inv;
                    }
                }
                cur_code = ci;
                // STG: the metadata must not be waited for again inside the frame
                // loop, where such a wait would also stall on the staged loads
                if constexpr (STG) vmem_wait_all();
            }
        }

        // -- frame set-up: gamma/mu, invalid-input check ----------------------
        if constexpr (VPT > 0) {
#pragma unroll
            for (int t = 0; t < VPT; ++t) {
                const int i = tid + t * NT;
                float g = 0.0f;
                if (i < C.n) g = gam[C.var_identity ? i : C.var_orig[i]];
                vg[t] = g * ip.mu_inv;
            }
        } else if constexpr (PERSIST) {
            if (!C.var_identity) {
                for (int i = tid; i < C.n; i += NT) gmu_row[i] = gam[C.var_orig[i]] * ip.mu_inv;
                __syncthreads();  // global staging, read by other threads in phase B
            }
        }
        if constexpr (PERSIST) {
            if (frame_invalid(fb, f)) {
                for (int i = tid; i < C.n; i += NT)
                    fb.x_out[(fb.x_off ? fb.x_off[f] : (int64_t)f * C.n) + i] = 0.5f;
                __syncthreads();
                if (tid == 0) {
                    fb.iters_out[f] = 0;
                    fb.flags_out[f] = 0x80;
                    if (fb.done) {
                        __threadfence_system();
                        __hip_atomic_store(fb.done + f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    }
                }
                __syncthreads();
                continue;
            }
        }

        // state location in global memory (non-resident forms)
        void *gz = nullptr;
        void *gu = nullptr;
        if constexpr (!RES) {
            const size_t base = PERSIST ? (size_t)blockIdx.x * state_stride : (size_t)f * C.E_int;
            gz = HALF ? (void *)(static_cast<__half *>(sa.z) + base) : (void *)(static_cast<float *>(sa.z) + base);
            gu = HALF ? (void *)(static_cast<__half *>(sa.u) + base) : (void *)(static_cast<float *>(sa.u) + base);
        }

        // -- initial state (PERSIST forms; the streamed form is initialised by
        //    its own kernel) -----------------------------------------------------
        if constexpr (PERSIST) {
            const size_t sbase = (size_t)f * C.E;
            if constexpr (RES) {
#pragma unroll
                for (int k = 0; k < CPT; ++k)
#pragma unroll
                    for (int e = 0; e < DMAX; ++e) {
                        float z0 = 0.0f, u0 = 0.0f;
                        if (sio.z_in && cval[k] && e < cdeg[k]) {
                            const int ce = csr_row(C.edge_csr, coff[k] + e * kWave)[lane];
                            z0 = sio.z_in[sbase + ce];
                            u0 = sio.u_in[sbase + ce];
                        }
                        z[k][e] = z0;
                        u[k][e] = u0;
                    }
            } else {
                for (int c = wave; c < C.nchunks && wave < C.waves; c += C.waves) {
                    const ChunkDesc h = chunk_desc(C, c);
                    const int d = h.deg, off = h.off;
                    const bool lv = lane < h.cnt;
                    for (int e = 0; e < d; ++e) {
                        const int p = off + e * kWave + lane;
                        float z0 = 0.0f, u0 = 0.0f;
                        if (sio.z_in && lv) {
                            const int ce = C.edge_csr[p];
                            z0 = sio.z_in[sbase + ce];
                            u0 = sio.u_in[sbase + ce];
                        }
                        st_state<HALF>(gz, p, z0);
                        st_state<HALF>(gu, p, u0);
                    }
                }
            }
        }

        if constexpr (SM == 2) {  // fresh accumulators (and previous x) for this frame
            for (int i = tid; i < C.n; i += NT) {
                acc[i] = 0ull;
                if (xprev) xprev[i] = 0u;
            }
            wg_barrier<LBAR>();
        }

        // -- phases ---------------------------------------------------------
        auto phase_a = [&]() {
            if constexpr (CPT > 0) {
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if constexpr (STG) {
#pragma unroll
                        for (int e = 0; e < DMAX; ++e) {
                            if (cval[k] && e < cdeg[k]) {
                                const int p = coff[k] + e * kWave + lane;
                                z[k][e] = stg_z[p];
                                u[k][e] = stg_u[p];
                            }
                        }
                    } else if constexpr (!RES) {
#pragma unroll
                        for (int e = 0; e < DMAX; ++e) {
                            if (cval[k] && e < cdeg[k]) {
                                const size_t p = coff[k] + e * kWave + lane;
                                z[k][e] = ld_state<HALF>(gz, p);
                                u[k][e] = ld_state<HALF>(gu, p);
                            }
                        }
                    }
                    if constexpr (MREG) {
                        if (cval[k]) {  // one lane mask per chunk; all-degree-6 codes need no per-edge test
#pragma unroll
                            for (int e = 0; e < DMAX; ++e)
                                if (DMIN == DMAX || e < cdeg[k]) slots[meta[k][e] >> 16] = z[k][e] - u[k][e];
                        }
                    } else {
                        uint32_t mt[DMAX];
                        load_meta<DMAX>(mt, opaque_ptr(C.edge_meta), coff[k], cdeg[k], lane);
                        if (cval[k]) {
#pragma unroll
                            for (int e = 0; e < DMAX; ++e)
                                if (e < cdeg[k]) slots[mt[e] >> 16] = z[k][e] - u[k][e];
                        }
                    }
                }
            } else {
                for (int c = wave; c < C.nchunks && wave < C.waves; c += C.waves) {
                    const ChunkDesc h = chunk_desc(C, c);
                    if (lane < h.cnt) {
                        if constexpr (DMIN == DMAX || !PERSIST) {
                            // the degree as a constant: all of the chunk's loads are
                            // issued before the first is used
                            dispatch_degree<DMIN, DMAX>(h.deg, [&](auto dc) {
                                constexpr int D = decltype(dc)::value;
                                float w[D];
                                uint32_t mt[D];
#pragma unroll
                                for (int e = 0; e < D; ++e) {
                                    const size_t p = h.off + e * kWave + lane;
                                    w[e] = ld_state<HALF>(gz, p) - ld_state<HALF>(gu, p);
                                    mt[e] = as_global(SM == 2 ? C.edge_acc : C.edge_meta)[p];
                                }
#pragma unroll
                                for (int e = 0; e < D; ++e) {
                                    if constexpr (SM == 2) atomicAdd(acc_entry(acc, mt[e]), to_fixed(w[e]));
                                    else slots[mt[e] >> 16] = w[e];
                                }
                            });
                        } else {  // persistent 2..8 kernel: the seven copies measured slower
                            for (int e = 0; e < h.deg; ++e) {
                                const size_t p = h.off + e * kWave + lane;
                                const float w = ld_state<HALF>(gz, p) - ld_state<HALF>(gu, p);
                                const uint32_t mt = as_global(SM == 2 ? C.edge_acc : C.edge_meta)[p];
                                if constexpr (SM == 2) atomicAdd(acc_entry(acc, mt), to_fixed(w));
                                else slots[mt >> 16] = w;
                            }
                        }
                    }
                }
            }
        };

        auto phase_b = [&]() {
            // the thread index through an empty asm: the per-thread address arithmetic of
            // this phase is then formed here each time instead of being hoisted to the
            // kernel's start, where its values stayed live and spilled to scratch
            int tb = tid;
            asm volatile("" : "+v"(tb));
            if constexpr (VPT > 0 && DV > 0) {
                constexpr float inv = 1.0f / (float)DV;
#pragma unroll
                for (int t = 0; t < VPT; ++t) {
                    const int i = tid + t * NT;
                    if (i < C.n) {
                        float acc = 0.0f;
#pragma unroll
                        for (int p = 0; p < DV; ++p) acc += slots[DV * i + p];
                        xs[i] = clamp01((acc - vg[t]) * inv);
                    }
                }
            } else if constexpr (VPT > 0) {
#pragma unroll
                for (int t = 0; t < VPT; ++t) {
                    const int i = tid + t * NT;
                    if (i < C.n) xs[i] = x_update(slots, VarLoc{vslot[t], vdeg[t], vinv[t]}, vg[t]);
                }
            } else if constexpr (SM == 2) {
                // the persistent forms keep the previous x in xprev; the streamed form's
                // entries start each launch with a zero high word
                acc_x_update<4, PERSIST>(acc, xprev, C.var_identity ? gam : gmu_row,
                                         C.var_identity ? ip.mu_inv : 1.0f, C, tid, NT);
            } else {
                // gamma/mu: straight from the frame's LLRs when variables keep their
                // order, else from the copy staged in internal order
                const auto gsrc = as_global(C.var_identity ? gam : gmu_row);
                const float gscale = C.var_identity ? ip.mu_inv : 1.0f;
                if constexpr (STG) {  // gamma/mu taken from the staging area in phase A
#pragma unroll
                    for (int t = 0; t < GQ; ++t) {
                        const int i = tb + t * NT;
                        if (i < C.n) {
                            const int b = C.dv * i;
                            float acc = 0.0f;
                            for (int p = 0; p < C.dv; ++p) acc += slots[b + p];
                            xs[i] = clamp01((acc - gq[t]) * C.dv_inv);
                        }
                    }
                } else if (C.dv > 0) {  // kernel-uniform degree: four variables per pass, loads first
                    for (int i0 = tb; i0 < C.n; i0 += 4 * NT) {
                        float g[4];
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int i = i0 + t * NT;
                            g[t] = (i < C.n) ? gsrc[i] : 0.0f;
                        }
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int i = i0 + t * NT;
                            if (i < C.n) {
                                const int b = C.dv * i;
                                float acc = 0.0f;
                                for (int p = 0; p < C.dv; ++p) acc += slots[b + p];
                                xs[i] = clamp01((acc - g[t] * gscale) * C.dv_inv);
                            }
                        }
                    }
                } else {  // mixed degrees: one degree class at a time
                    // Variables are numbered by decreasing degree, so a class is a range
                    // of variables with one degree and consecutive slot blocks: the
                    // degree is a constant for the class's sums (degrees up to 8; larger
                    // ones sum in a loop) and a variable's block follows from its index.
                    // Sums run over the block in slot order, as x_update does.
                    for (int c = 0; c < C.nvc; ++c) {  // wave-uniform
                        const int b = C.vc_start[c], end = C.vc_start[c + 1], deg = C.vc_deg[c];
                        const int s0 = C.vc_slot0[c];
                        const float inv = C.vc_inv[c];
                        auto sums = [&](auto dc) {
                            constexpr int DVC = decltype(dc)::value;
                            constexpr int VC = 2;  // variables per pass
                            for (int i0 = b + tb; i0 < end; i0 += VC * NT) {
                                float g[VC];
#pragma unroll
                                for (int t = 0; t < VC; ++t) {
                                    const int i = i0 + t * NT;
                                    g[t] = (i < end) ? gsrc[i] : 0.0f;
                                }
#pragma unroll
                                for (int t = 0; t < VC; ++t) {
                                    const int i = i0 + t * NT;
                                    if (i < end) {
                                        const int sb = s0 + (i - b) * deg;
                                        float a = 0.0f;
                                        if constexpr (DVC > 0) {
#pragma unroll
                                            for (int p = 0; p < DVC; ++p) a += slots[sb + p];
                                        } else {
                                            for (int p = 0; p < deg; ++p) a += slots[sb + p];
                                        }
                                        xs[i] = clamp01((a - g[t] * gscale) * inv);
                                    }
                                }
                            }
                        };
                        if (deg >= 1 && deg <= 8) dispatch_degree<1, 8>(deg, sums);
                        else sums(std::integral_constant<int, 0>{});
                    }
                }
            }
        };

        auto phase_c = [&](float &rp, float &rd) {
            if constexpr (CPT > 0 && !MREG) {
                // metadata read from memory, one chunk ahead of its use; each chunk's
                // slot writes for the next iteration follow its update, reusing it
                // (the table pointer is made opaque so that the loads stay in the
                // iteration instead of being hoisted out of it into registers)
                const uint32_t *em = opaque_ptr(C.edge_meta);
                uint32_t mcur[DMAX], mnext[DMAX];
                load_meta<DMAX>(mcur, em, coff[0], cdeg[0], lane);
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (k + 1 < CPT) load_meta<DMAX>(mnext, em, coff[k + 1], cdeg[k + 1], lane);
                    if (cdeg[k] != 0 && cval[k]) {  // cdeg wave-uniform
                        dispatch_degree<DMIN, DMAX>(cdeg[k], [&](auto dc) {
                            constexpr int D = decltype(dc)::value;
                            check_update<D, XS>(z[k], u[k], mcur, xs, ip.rho, rp, rd);
                            if constexpr (FUSED_A) {
#pragma unroll
                                for (int e = 0; e < D; ++e) slots[mcur[e] >> 16] = z[k][e] - u[k][e];
                            }
                        });
                    }
#pragma unroll
                    for (int e = 0; e < DMAX; ++e) mcur[e] = mnext[e];
                }
            } else if constexpr (CPT > 0) {
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (cdeg[k] == 0) continue;  // wave-uniform
                    if (cval[k]) {
                        dispatch_degree<DMIN, DMAX>(cdeg[k], [&](auto dc) {
                            constexpr int D = decltype(dc)::value;
                            check_update<D, XS>(z[k], u[k], meta[k], xs, ip.rho, rp, rd);
                            if constexpr (FUSED_A) {
#pragma unroll
                                for (int e = 0; e < D; ++e) slots[meta[k][e] >> 16] = z[k][e] - u[k][e];
                            }
                        });
                    }
                    if constexpr (!RES) {
#pragma unroll
                        for (int e = 0; e < DMAX; ++e) {
                            if (cval[k] && e < cdeg[k]) {
                                const size_t p = coff[k] + e * kWave + lane;
                                st_state<HALF>(gz, p, z[k][e]);
                                st_state<HALF>(gu, p, u[k][e]);
                            }
                        }
                    }
                }
            } else {
                for (int c = wave; c < C.nchunks && wave < C.waves; c += C.waves) {
                    const ChunkDesc h = chunk_desc(C, c);
                    const int d = h.deg, off = h.off;
                    if (lane < h.cnt) {
                        dispatch_degree<DMIN, DMAX>(d, [&](auto dc) {
                            constexpr int D = decltype(dc)::value;
                            float zz[D], uu[D];
                            uint32_t mm[D];
#pragma unroll
                            for (int e = 0; e < D; ++e) {
                                const size_t p = off + e * kWave + lane;
                                zz[e] = ld_state<HALF>(gz, p);
                                uu[e] = ld_state<HALF>(gu, p);
                                mm[e] = as_global(SM == 2 ? C.edge_acc : C.edge_meta)[p];
                            }
                            check_update<D, XS, SM == 2>(zz, uu, mm, xs, ip.rho, rp, rd);
#pragma unroll
                            for (int e = 0; e < D; ++e) {
                                const size_t p = off + e * kWave + lane;
                                st_state<HALF>(gz, p, zz[e]);
                                st_state<HALF>(gu, p, uu[e]);
                            }
                        });
                    }
                }
            }
        };

        auto publish = [&](int buf, float rp, float rd) {
            rp = wave_sum(rp);
            rd = wave_sum(rd);
            if (lane == 0) {
                s_red[buf][0][wave] = rp;
                s_red[buf][1][wave] = rd;
            }
        };
        auto converged = [&](int buf) -> bool {  // identical result in every wave
            const float a = lane < NW ? s_red[buf][0][lane] : 0.0f;
            const float b = lane < NW ? s_red[buf][1][lane] : 0.0f;
            return row0_sum(a) < thr && row0_sum(b) < thr;
        };

        int iters;
        bool conv = false;
        if constexpr (PERSIST) {
            // iteration it = B, C, then the next iteration's A; the stopping test
            // for it reads the residuals published by C after the barrier that
            // follows that A, so it costs no barrier of its own
            int it = 1;
            phase_a();
            wg_barrier<LBAR>();
            for (;; ++it) {
                phase_b();
                wg_barrier<LBAR>();
                float rp = 0.0f, rd = 0.0f;
                phase_c(rp, rd);
                publish(it & 1, rp, rd);
                // accumulator mode: the next phase A adds into the entries that
                // phase C is still reading x from
                if constexpr (SM == 2) wg_barrier<LBAR>();
                if constexpr (!FUSED_A) phase_a();  // else done chunk by chunk in phase C
                wg_barrier<LBAR>();
                if (__builtin_amdgcn_readfirstlane(converged(it & 1))) { conv = true; break; }
                if (it >= ip.max_iter) break;
            }
            iters = conv ? it : ip.max_iter;
            if constexpr (SM == 2) {
                // The stopping test ran after the next iteration's phase A, which
                // accumulated into the entries holding x: restore the last x.
                for (int i = tid; i < C.n; i += NT) acc[i] = (unsigned long long)xprev[i] << 32;
                __syncthreads();
            }
        } else {
            const int it = iter0 + 1;
            auto pbar = [&]() {
                if constexpr (STG) lds_barrier_nofence();
                else wg_barrier<LBAR>();
            };
            if constexpr (STG) {
                const float gscale = C.var_identity ? ip.mu_inv : 1.0f;
#pragma unroll
                for (int t = 0; t < GQ; ++t) {
                    const int i = tid + t * NT;
                    gq[t] = (i < C.n) ? stg_g[i] * gscale : 0.0f;
                }
            }
            phase_a();
            pbar();
            if constexpr (STG) {
                // every wave has read the staged frame: stage the next one
                const int g = next_active();
                pending = g;
                if (g < fb.nframes) stage_issue(C, g);
            }
            phase_b();
            pbar();
            float rp = 0.0f, rd = 0.0f;
            phase_c(rp, rd);
            publish(0, rp, rd);
            pbar();
            conv = converged(0);
            iters = it;
            const bool fin = __builtin_amdgcn_readfirstlane(conv || it >= ip.max_iter);
            if (tid == 0) {
                sa.st[f].iter = it;
                if (fin) sa.st[f].done = 1;
                else list_unfinished(f);
            }
            if (!fin) {
                pbar();  // LDS reuse by the next frame of this workgroup
                continue;
            }
        }

        // -- epilogue: x, iteration count and certificate flags (x in LDS) ---------
        const int64_t xoff = fb.x_off ? uniform_i64(fb.x_off[f]) : (int64_t)f * C.n;
        float frac = 0.0f;
        for (int i = tid; i < C.n; i += NT) {
            const float x = xs[XS * i];
            fb.x_out[xoff + (C.var_identity ? i : C.var_orig[i])] = x;
            frac = fmaxf(frac, fminf(x, 1.0f - x));
        }
        bool odd = false;
        for (int c = wave; c < C.nchunks && wave < C.waves; c += C.waves) {
            const ChunkDesc h = chunk_desc(C, c);
            const int d = h.deg, off = h.off;
            if (lane < h.cnt) {
                bool par = false;
                for (int e = 0; e < d; ++e)
                    par ^= (xs[XS * (C.edge_meta[off + e * kWave + lane] & 0xffffu)] >= 0.5f);
                odd |= par;
            }
        }
        // frac > 1e-3 exactly: 1e-3f is the least float above 1e-3
        const bool nonint = frac >= 1e-3f;
        const int any_odd = __syncthreads_or(odd);
        const int any_nonint = __syncthreads_or(nonint);
        if (tid == 0) {
            uint8_t fl = conv ? 0x01 : 0x00;
            if (!any_nonint) fl |= 0x02;
            if (!any_odd) fl |= 0x04;
            if ((fl & 0x07) == 0x07) fl |= 0x08;
            fb.iters_out[f] = iters;
            fb.flags_out[f] = fl;
            if (fb.done) {
                // every thread's x store precedes the barrier above; publish them
                // to the host before the completion flag
                __threadfence_system();
                __hip_atomic_store(fb.done + f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        // state export (CSR edge order)
        if (sio.z_out) {
            const size_t sbase = (size_t)f * C.E;
            if constexpr (RES) {
#pragma unroll
                for (int k = 0; k < CPT; ++k)
#pragma unroll
                    for (int e = 0; e < DMAX; ++e)
                        if (cval[k] && e < cdeg[k]) {
                            const int ce = csr_row(C.edge_csr, coff[k] + e * kWave)[lane];
                            sio.z_out[sbase + ce] = z[k][e];
                            sio.u_out[sbase + ce] = u[k][e];
                        }
            } else {
                for (int c = wave; c < C.nchunks && wave < C.waves; c += C.waves) {
                    const ChunkDesc h = chunk_desc(C, c);
                    const int d = h.deg, off = h.off;
                    if (lane < h.cnt) {
                        for (int e = 0; e < d; ++e) {
                            const size_t p = off + e * kWave + lane;
                            const int ce = C.edge_csr[p];
                            sio.z_out[sbase + ce] = ld_state<HALF>(gz, p);
                            sio.u_out[sbase + ce] = ld_state<HALF>(gu, p);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Two frames per workgroup: the register-resident form for codes whose checks
// all have degree 6 and whose variables all have degree 3, planned with two
// chunks per wave.
//
// A CU deals the waves of a workgroup to its 4 SIMDs in turn, so waves w, w+4,
// w+8 share a SIMD, and the check phase of an iteration lasts as long as the
// SIMD that holds the most chunks: one frame of 21 chunks on 11 waves gives its
// SIMDs 6, 6, 5 and 4.  Here a workgroup of 12 waves holds two frames
// ("slots").  The code's plan of W waves (wave v owns chunks v and v + W) is kept
// as W virtual waves per slot; each physical wave hosts at most one virtual wave
// of each slot, in an assignment made on the host to even out the chunks per
// SIMD (21 chunks: 11, 11, 10, 10 for two frames instead of 12).  A virtual wave
// forms its residual sums exactly as a wave of the one-frame kernel does, and
// the stopping test adds them in virtual-wave order, so results are bitwise the
// same.
//
// The iteration loop runs both slots in step (x-updates, barrier, check updates,
// barrier, two stopping tests).  Only when a frame stops does the workgroup
// leave it: it writes that frame's x, flags and state, takes the next frame
// from the queue, sets it up and rejoins the loop, while the other slot waits.
// Once the queue is empty the remaining frame finishes in a one-slot loop.
// ---------------------------------------------------------------------------
constexpr int kPairWaves = 12;
constexpr int kPairNone = 0xF;  // no virtual wave (4-bit field of the assignment)

template <int VPT>
__global__ void __launch_bounds__(kPairWaves * kWave, 1)
k_decode_pair(const DevCode *__restrict__ codes, FrameBatch fb, IterParams ip, StateIO sio,
              unsigned long long host0, unsigned long long host1, int lds_E) {
    constexpr int D = 6, DV = 3, NT = kPairWaves * kWave;
    constexpr float inv = 1.0f / (float)DV;
    extern __shared__ __attribute__((aligned(16))) float lds[];
    __shared__ float s_red[2][2][kMaxWaves];
    __shared__ int s_frame[2];
    __shared__ int s_vote[2][kPairWaves];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const DevCode &C = codes[0];
    const int W = C.waves;
    const int region = lds_E + C.n;  // per slot: slots [lds_E], then x [n]
    const float thr = ip.tol2 * (float)C.E;
    const bool lw = lane < W;

    // virtual wave of each slot hosted by this wave (-1: none); chunk k of this
    // wave is chunk vw[k >> 1] + (k & 1) W of the code
    int vw[2];
    {
        const int a = (int)((host0 >> (4 * wave)) & 0xFull), b = (int)((host1 >> (4 * wave)) & 0xFull);
        vw[0] = a == kPairNone ? -1 : a;
        vw[1] = b == kPairNone ? -1 : b;
    }
    float z[4][D], u[4][D];
    uint32_t meta[4][D];
    int coff[4];
    int cpres = 0;  // bit k: chunk k exists (wave-uniform)
    bool cval[4];   // this lane's check of chunk k exists
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int v = vw[k >> 1];
        const int c = v + (k & 1) * W;
        const bool has = v >= 0 && c < C.nchunks;
        const ChunkDesc h = has ? chunk_desc(C, c) : ChunkDesc{0, 0, 0};
        if (has) cpres |= 1 << k;
        coff[k] = h.off;
        cval[k] = lane < h.cnt;
#pragma unroll
        for (int e = 0; e < D; ++e) meta[k][e] = cval[k] ? C.edge_meta[h.off + e * kWave + lane] : 0u;
    }
    float vg[2][VPT];

    // -- the iteration's phases for slot s --------------------------------------
    auto phase_b = [&](auto sc) {
        constexpr int s = decltype(sc)::value;
        const float *slots = lds + s * region;
        float *xs = lds + s * region + lds_E;
#pragma unroll
        for (int t = 0; t < VPT; ++t) {
            const int i = tid + t * NT;
            if (i < C.n) {
                float acc = 0.0f;
#pragma unroll
                for (int p = 0; p < DV; ++p) acc += slots[DV * i + p];
                xs[i] = clamp01((acc - vg[s][t]) * inv);
            }
        }
    };
    auto phase_c = [&](auto sc) {  // check updates, the next iteration's slot writes, residuals
        constexpr int s = decltype(sc)::value;
        float *slots = lds + s * region;
        const float *xs = lds + s * region + lds_E;
        float rp = 0.0f, rd = 0.0f;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = 2 * s + j;
            if (!(cpres & (1 << k))) continue;  // wave-uniform
            if (cval[k]) {
                check_update<D>(z[k], u[k], meta[k], xs, ip.rho, rp, rd);
#pragma unroll
                for (int e = 0; e < D; ++e) slots[meta[k][e] >> 16] = z[k][e] - u[k][e];
            }
        }
        if (vw[s] >= 0) {
            rp = wave_sum(rp);
            rd = wave_sum(rd);
            if (lane == 0) {
                s_red[s][0][vw[s]] = rp;
                s_red[s][1][vw[s]] = rd;
            }
        }
    };
    auto converged = [&](int s) -> bool {  // identical result in every wave
        const float a = lw ? s_red[s][0][lane] : 0.0f;
        const float b = lw ? s_red[s][1][lane] : 0.0f;
        return __builtin_amdgcn_readfirstlane(row0_sum(a) < thr && row0_sum(b) < thr);
    };

    // -- frame changes ---------------------------------------------------------
    // The next valid frame for slot s (>= nframes: the queue is empty).  With
    // `fetched`, thread 0 took its queue position into s_frame[s] before the last
    // barrier (when the previous frame stopped, so that the queue's latency hides
    // behind writing that frame's x).  Frames with a non-finite LLR are completed
    // on the way (x = 1/2, flags 0x80) and replaced from the queue.
    auto frame_at = [&](int q) { return (fb.order && q < fb.nframes) ? fb.order[q] : q; };
    auto acquire = [&](int s, bool fetched) -> int {
        for (;;) {
            if (!fetched) {
                if (tid == 0) s_frame[s] = frame_at(atomicAdd(fb.queue, 1));
                __syncthreads();
            }
            fetched = false;
            const int f = __builtin_amdgcn_readfirstlane(s_frame[s]);
            if (f >= fb.nframes || !frame_invalid(fb, f)) return f;
            for (int i = tid; i < C.n; i += NT) fb.x_out[(fb.x_off ? fb.x_off[f] : (int64_t)f * C.n) + i] = 0.5f;
            __syncthreads();  // also: every wave has read s_frame[s] before the next fetch
            if (tid == 0) {
                fb.iters_out[f] = 0;
                fb.flags_out[f] = 0x80;
                if (fb.done) {
                    __threadfence_system();
                    __hip_atomic_store(fb.done + f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
        }
    };
    // gamma/mu and the state of frame f, then its slot writes (phase A)
    auto setup = [&](auto sc, int f) {
        constexpr int s = decltype(sc)::value;
        float *slots = lds + s * region;
        const float *gam = fb.llr + (fb.llr_off ? fb.llr_off[f] : (int64_t)f * C.n);
#pragma unroll
        for (int t = 0; t < VPT; ++t) {
            const int i = tid + t * NT;
            float g = 0.0f;
            if (i < C.n) g = gam[C.var_identity ? i : C.var_orig[i]];
            vg[s][t] = g * ip.mu_inv;
        }
        const size_t sbase = (size_t)f * C.E;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = 2 * s + j;
#pragma unroll
            for (int e = 0; e < D; ++e) {
                float z0 = 0.0f, u0 = 0.0f;
                if (sio.z_in && cval[k]) {
                    const int ce = C.edge_csr[coff[k] + e * kWave + lane];
                    z0 = sio.z_in[sbase + ce];
                    u0 = sio.u_in[sbase + ce];
                }
                z[k][e] = z0;
                u[k][e] = u0;
            }
            if (cval[k]) {
#pragma unroll
                for (int e = 0; e < D; ++e) slots[meta[k][e] >> 16] = z[k][e] - u[k][e];
            }
        }
    };
    // x, the parity votes and the state of the finished frame f
    auto finish_x = [&](auto sc, int f) {
        constexpr int s = decltype(sc)::value;
        const float *xs = lds + s * region + lds_E;
        const int64_t xoff = fb.x_off ? uniform_i64(fb.x_off[f]) : (int64_t)f * C.n;
        float frac = 0.0f;
        for (int i = tid; i < C.n; i += NT) {
            const float x = xs[i];
            fb.x_out[xoff + (C.var_identity ? i : C.var_orig[i])] = x;
            frac = fmaxf(frac, fminf(x, 1.0f - x));
        }
        // parity of this wave's checks of slot s (the virtual waves cover every chunk once)
        bool odd = false;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = 2 * s + j;
            if (cval[k]) {
                bool par = false;
#pragma unroll
                for (int e = 0; e < D; ++e) par ^= (xs[meta[k][e] & 0xffffu] >= 0.5f);
                odd |= par;
            }
        }
        // frac > 1e-3 exactly: 1e-3f is the least float above 1e-3
        const bool nonint = frac >= 1e-3f;
        const int vote = (__ballot(odd) ? 1 : 0) | (__ballot(nonint) ? 2 : 0);
        if (lane == 0) s_vote[s][wave] = vote;
        if (sio.z_out) {
            const size_t sbase = (size_t)f * C.E;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int k = 2 * s + j;
                if (cval[k]) {
#pragma unroll
                    for (int e = 0; e < D; ++e) {
                        const int ce = C.edge_csr[coff[k] + e * kWave + lane];
                        sio.z_out[sbase + ce] = z[k][e];
                        sio.u_out[sbase + ce] = u[k][e];
                    }
                }
            }
        }
    };
    // Barrier between finish_x and finish_flags: the votes go through LDS; with
    // host-visible completion flags the x and state stores must also have landed
    // before a flag is raised, which a full barrier waits for.
    auto flags_barrier = [&]() {
        if (fb.done) __syncthreads();
        else wg_barrier<true>();
    };
    // its iteration count and flags, after flags_barrier
    auto finish_flags = [&](int s, int f, int iters, bool conv) {
        if (tid == 0) {
            int any_odd = 0, any_nonint = 0;
            for (int w = 0; w < kPairWaves; ++w) {
                any_odd |= s_vote[s][w] & 1;
                any_nonint |= s_vote[s][w] & 2;
            }
            uint8_t fl = conv ? 0x01 : 0x00;
            if (!any_nonint) fl |= 0x02;
            if (!any_odd) fl |= 0x04;
            if ((fl & 0x07) == 0x07) fl |= 0x08;
            fb.iters_out[f] = iters;
            fb.flags_out[f] = fl;
            if (fb.done) {
                __threadfence_system();
                __hip_atomic_store(fb.done + f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    };

    constexpr std::integral_constant<int, 0> S0{};
    constexpr std::integral_constant<int, 1> S1{};
    int f0 = acquire(0, false), f1 = acquire(1, false);
    bool live0 = f0 < fb.nframes, live1 = f1 < fb.nframes;
    if (live0) setup(S0, f0);
    if (live1) setup(S1, f1);
    wg_barrier<true>();
    int it0 = 1, it1 = 1;
    if (live0 && live1) {
        for (;;) {
            phase_b(S0);
            phase_b(S1);
            wg_barrier<true>();
            phase_c(S0);
            __builtin_amdgcn_sched_barrier(0);  // the two slots' updates one after the other
            phase_c(S1);
            wg_barrier<true>();
            const bool c0 = converged(0), c1 = converged(1);
            const bool stop0 = c0 || it0 >= ip.max_iter, stop1 = c1 || it1 >= ip.max_iter;
            if (!stop0 && !stop1) {
                ++it0;
                ++it1;
                continue;
            }
            // a frame has stopped: fetch the next one's index, finish it, start the next
            // one.  Near the end of the queue (fewer frames left than workgroups) a slot
            // whose partner keeps running takes no new frame: the workgroup then runs one
            // frame at a time, each at the one-frame rate, so that the last frames do not
            // run at the shared rate while other CUs have nothing left.  The partner's
            // one-slot loop keeps taking frames, so none is left behind.
            if (tid == 0) {
                const bool late = __hip_atomic_load(fb.queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                                  fb.nframes - (int)gridDim.x;
                if (stop0) s_frame[0] = (late && !stop1) ? fb.nframes : frame_at(atomicAdd(fb.queue, 1));
                if (stop1) s_frame[1] = late ? fb.nframes : frame_at(atomicAdd(fb.queue, 1));
            }
            if (stop0) finish_x(S0, f0);
            if (stop1) finish_x(S1, f1);
            flags_barrier();
            if (stop0) finish_flags(0, f0, c0 ? it0 : ip.max_iter, c0);
            if (stop1) finish_flags(1, f1, c1 ? it1 : ip.max_iter, c1);
            if (!stop0) ++it0;
            if (!stop1) ++it1;
            if (stop0) {
                f0 = acquire(0, true);
                live0 = f0 < fb.nframes;
                if (live0) {
                    setup(S0, f0);
                    it0 = 1;
                }
            }
            if (stop1) {
                f1 = acquire(1, true);
                live1 = f1 < fb.nframes;
                if (live1) {
                    setup(S1, f1);
                    it1 = 1;
                }
            }
            wg_barrier<true>();  // the new frames' slot writes precede the x-update
            if (!live0 || !live1) break;
        }
    }
    // the queue is empty: the remaining frame (if any) finishes alone
    auto tail = [&](auto sc, int f, int it) {
        constexpr int s = decltype(sc)::value;
        for (;;) {
            phase_b(sc);
            wg_barrier<true>();
            phase_c(sc);
            wg_barrier<true>();
            const bool c = converged(s);
            if (!(c || it >= ip.max_iter)) {
                ++it;
                continue;
            }
            if (tid == 0) s_frame[s] = frame_at(atomicAdd(fb.queue, 1));
            finish_x(sc, f);
            flags_barrier();
            finish_flags(s, f, c ? it : ip.max_iter, c);
            f = acquire(s, true);
            if (f >= fb.nframes) break;
            setup(sc, f);
            it = 1;
            wg_barrier<true>();
        }
    };
    if (live0) tail(S0, f0, it0);
    else if (live1) tail(S1, f1, it1);
}

// ---------------------------------------------------------------------------
// Large codes whose checks all have one degree D and whose exchange goes through
// the LDS fixed-point accumulators (the slot array does not fit in LDS): the
// persistent-global and streamed forms with the first KR chunks of each wave held
// in registers from phase A to phase C.  k_decode's chunk walk reads a chunk's z, u
// in phase A (for the sums) and again in phase C (for the update); here a held
// chunk is read once per iteration (streamed form) or never leaves the registers
// while its frame runs (persistent-global form), and only a wave's chunks beyond
// the first KR are walked as before.  The arithmetic, the order of the residual
// sums and the exchange are those of k_decode, so results are bitwise the same.
// Chunks are padded to 64 lanes in every array, so a held chunk's rows are loaded
// for all lanes without a branch (padding lanes take no part in the update).
// FP16 storage in the persistent-global form keeps a held edge's z and u as two
// FP16 values in one register (z in the low half) and the walked chunks' state as
// FP16 in the workgroup's scratch; each update rounds z and u to FP16 as the
// streamed form's stores do, so the two forms' results are bitwise the same.  Half
// the registers per held chunk lets the (3,6) n = 16384 code hold all its chunks.
// VW = 2 (persistent-global, every chunk held): each hardware wave hosts two of the
// plan's waves (wave w and w + NW), so a workgroup of half the waves has twice the
// registers per wave and holds an FP32 frame of the (3,6) n = 16384 code whole.  The
// residuals are kept and published per plan wave, so the stopping test sums the same
// partial sums in the same order as with one plan wave per hardware wave.
template <int D, int KR, bool HALF, bool PERSIST, int VW = 1>
__global__ void __launch_bounds__(kMaxThreads / VW, 1)
k_decode_acc(const DevCode *__restrict__ codes, FrameBatch fb, IterParams ip, StateIO sio, StreamArgs sa,
             int state_stride) {
    static_assert(KR >= 0, "held chunks per wave");
    constexpr int KH = KR > 0 ? KR : 1;  // register arrays of the held chunks
    constexpr bool PK = HALF && PERSIST;  // held chunks as packed FP16 pairs
    // KR = kAccAllHeld: every chunk of a wave is held (the host launches it only for
    // codes of at most that many chunks per wave), and the chunk walk is compiled out
    constexpr bool WALK = KR < kAccAllHeld;
    static_assert(VW == 1 || (VW == 2 && PERSIST && !WALK), "two plan waves per wave: all chunks held");
    constexpr int NH = VW * KR;                // held chunks per hardware wave
    constexpr int NHA = NH > 0 ? NH : 1;
    // no static LDS (the launcher checks): the dynamic array starts at address 0, and
    // the accumulator atomics and x reads address LDS by the entries' byte offsets
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int NT = blockDim.x;
    const int NW = NT >> 6;
    const DevCode &C = codes[0];
    const int W = C.waves, cpt = C.cpt;  // the plan's waves (NW = W when VW = 1)
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(lds);
    const float *xs = lds_at<const float>(4);  // x sits in each accumulator's high word (stride 2)
    char *tail = reinterpret_cast<char *>(lds) + acc_tail_offset(C.n);
    float(*s_red)[2][kMaxWaves] = reinterpret_cast<float(*)[2][kMaxWaves]>(tail);
    int &s_frame = *reinterpret_cast<int *>(tail + kAccFrameOffset);
    int *s_vote = reinterpret_cast<int *>(tail + kAccVoteOffset);
    unsigned *xprev = PERSIST ? sa.gxprev + (size_t)blockIdx.x * sa.gmu_stride : nullptr;
    const float thr = ip.tol2 * (float)C.E;

    // held chunk h = j KH + k of this wave: chunk v + k W of plan wave v = wave + j NW
    // (a missing one repeats the wave's first chunk, whose lanes then take no part)
    int hoff[NHA];
    bool hval[NHA];
#pragma unroll
    for (int h = 0; h < NHA; ++h) {
        const int v = wave + (h / KH) * NW, k = h % KH;
        const int c = v + k * W;
        const bool has = v < W && k < cpt && c < C.nchunks;
        const ChunkDesc cd = chunk_desc(C, has ? c : wave);
        hoff[h] = cd.off;
        hval[h] = has && lane < cd.cnt;
    }
    float zr[PK ? 1 : NHA][D], ur[PK ? 1 : NHA][D];
    unsigned hr[PK ? NHA : 1][D];  // PK: z | u << 16 (FP16 bits) of held edge e of chunk h

    const int launch = PERSIST ? 0 : streamed_launch(ip, sa);
    // Streamed form: the frames still running after the previous launch, listed in
    // the order they finished it, are dealt to the workgroups in turn (entry
    // blockIdx.x + k G, G = gridDim.x), so every workgroup gets the same number of
    // frames to within one however few remain.  Each frame that stays unfinished
    // appends itself to this launch's list.
    // The list entries are read 64 at a time (one per lane, with their done flags)
    // and the unfinished frames taken from a ballot mask, identical in every wave.
    int lcnt = 0;
    const int *lprev = nullptr;
    if constexpr (!PERSIST) {
        lcnt = min(uniform_i32(sa.alist_cnt[(launch + 2) % 3]), fb.nframes);
        lprev = sa.alist + (size_t)((launch + 1) & 1) * fb.nframes;
        if (blockIdx.x == 0 && tid == 0) {
            sa.active_count[(launch + 1) & 1] = 0;  // next launch's counter
            sa.alist_cnt[(launch + 1) % 3] = 0;     // next launch's list
        }
    }
    int lbase = (int)blockIdx.x - kWave * (int)gridDim.x;
    int lframe = 0;  // this lane's frame of the current group of entries
    unsigned long long lmask = 0ull;
    auto next_active = [&]() -> int {
        for (;;) {
            if (lmask) {
                const int j = __builtin_ctzll(lmask);
                lmask &= lmask - 1ull;
                return __builtin_amdgcn_readlane(lframe, j);
            }
            lbase += kWave * (int)gridDim.x;
            if (lbase >= lcnt) return fb.nframes;
            const int lj = lbase + lane * (int)gridDim.x;
            const int g = lj < lcnt ? lprev[lj] : -1;
            lframe = g;
            lmask = __ballot(g >= 0 && g < fb.nframes && !sa.st[g].done);
        }
    };
    // a frame that stays unfinished: count it and list it for the next launch
    auto list_unfinished = [&](int g) {
        atomicAdd(sa.active_count + (launch & 1), 1);
        const int pos = atomicAdd(sa.alist_cnt + launch % 3, 1);
        if (pos < fb.nframes) sa.alist[(size_t)(launch & 1) * fb.nframes + pos] = g;
    };
    for (;;) {
        int f;
        if constexpr (PERSIST) {
            if (tid == 0) {
                const int q = atomicAdd(fb.queue, 1);
                s_frame = (fb.order && q < fb.nframes) ? fb.order[q] : q;
            }
            __syncthreads();
            f = __builtin_amdgcn_readfirstlane(s_frame);
            __syncthreads();
        } else {
            f = next_active();
        }
        if (f >= fb.nframes) break;
        const int64_t loff = fb.llr_off ? uniform_i64(fb.llr_off[f]) : (int64_t)f * C.n;
        const float *gam = fb.llr + loff;
        float *gmu_row = sa.gmu ? sa.gmu + (size_t)(PERSIST ? blockIdx.x : f) * sa.gmu_stride : nullptr;
        if constexpr (PERSIST) {
            if (!C.var_identity) {
                for (int i = tid; i < C.n; i += NT) gmu_row[i] = gam[C.var_orig[i]] * ip.mu_inv;
                __syncthreads();  // global staging, read by other threads in phase B
            }
            if (frame_invalid(fb, f)) {
                for (int i = tid; i < C.n; i += NT)
                    fb.x_out[(fb.x_off ? fb.x_off[f] : (int64_t)f * C.n) + i] = 0.5f;
                __syncthreads();
                if (tid == 0) {
                    fb.iters_out[f] = 0;
                    fb.flags_out[f] = 0x80;
                    if (fb.done) {
                        __threadfence_system();
                        __hip_atomic_store(fb.done + f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    }
                }
                __syncthreads();
                continue;
            }
        }
        const size_t sb = PERSIST ? (size_t)blockIdx.x * state_stride : (size_t)f * C.E_int;
        void *gz = HALF ? (void *)(static_cast<__half *>(sa.z) + sb) : (void *)(static_cast<float *>(sa.z) + sb);
        void *gu = HALF ? (void *)(static_cast<__half *>(sa.u) + sb) : (void *)(static_cast<float *>(sa.u) + sb);

        // initial state (persistent-global form; the streamed form has its own kernel):
        // held chunks in registers, walked chunks in the workgroup's scratch
        if constexpr (PERSIST) {
            const size_t fb0 = (size_t)f * C.E;
#pragma unroll
            for (int k = 0; k < NH; ++k)
#pragma unroll
                for (int e = 0; e < D; ++e) {
                    float z0 = 0.0f, u0 = 0.0f;
                    if (sio.z_in && hval[k]) {
                        // row address scalar, table pointer opaque: nothing per edge is
                        // hoisted out of the frame loop into registers
                        const int ce = csr_row(C.edge_csr, hoff[k] + e * kWave)[lane];
                        z0 = sio.z_in[fb0 + ce];
                        u0 = sio.u_in[fb0 + ce];
                    }
                    if constexpr (PK) {
                        hr[k][e] = pack_h2(z0, u0);
                    } else {
                        zr[k][e] = z0;
                        ur[k][e] = u0;
                    }
                }
            for (int k = KR; k < cpt; ++k) {
                const int c = wave + k * W;
                if (c >= C.nchunks) break;
                const ChunkDesc h = chunk_desc(C, c);
                for (int e = 0; e < D; ++e) {
                    const int p = h.off + e * kWave + lane;
                    float z0 = 0.0f, u0 = 0.0f;
                    if (sio.z_in && lane < h.cnt) {
                        const int ce = C.edge_csr[p];
                        z0 = sio.z_in[fb0 + ce];
                        u0 = sio.u_in[fb0 + ce];
                    }
                    st_state<HALF>(gz, p, z0);
                    st_state<HALF>(gu, p, u0);
                }
            }
        }
        // fresh accumulators (and previous x) for this frame
        for (int i = tid; i < C.n; i += NT) {
            acc[i] = 0ull;
            if constexpr (PERSIST) as_global_rw(xprev)[i] = 0u;
        }
        wg_barrier<true>();

        // A: the replica differences z - u into the accumulators
        // streamed form: this frame's z, u of held chunk k into its registers
        auto load_held = [&](int k) {
#pragma unroll
            for (int e = 0; e < D; ++e) {
                const size_t p = hoff[k] + e * kWave + lane;
                zr[k][e] = ld_state<HALF>(gz, p);
                ur[k][e] = ld_state<HALF>(gu, p);
            }
        };
        // the walked chunks k >= KR of this wave (chunk wave + k W), one chunk ahead:
        // chunk k + 1's z, u and metadata are loaded before chunk k is used, so a
        // wave keeps two chunks' loads in flight (all lanes load; padding lanes of a
        // chunk exist in every array and take no part)
        struct Walk {
            int k, off, cnt;
            bool has;
        };
        auto walk_at = [&](int k) -> Walk {
            const int c = wave + k * W;
            const bool has = k < cpt && c < C.nchunks;  // wave-uniform
            const ChunkDesc h = has ? chunk_desc(C, c) : ChunkDesc{0, 0, 0};
            return Walk{k, h.off, h.cnt, has};
        };
        auto walk_load = [&](const Walk &w, float *zz, float *uu, uint32_t *mm) {
#pragma unroll
            for (int e = 0; e < D; ++e) {
                const size_t p = w.off + e * kWave + lane;
                zz[e] = ld_state<HALF>(gz, p);
                uu[e] = ld_state<HALF>(gu, p);
                mm[e] = as_global(C.edge_acc)[p];
            }
        };
        auto phase_a = [&]() {
            if constexpr (KR > 0) {
                // held chunks, one ahead: chunk k + 1's loads are issued before chunk
                // k's accumulation waits for its own
                uint32_t mcur[D], mnext[D];
                if constexpr (!PERSIST) load_held(0);
                load_meta<D>(mcur, C.edge_acc, hoff[0], D, lane);
#pragma unroll
                for (int k = 0; k < NH; ++k) {
                    if (k + 1 < NH) {
                        if constexpr (!PERSIST) load_held(k + 1);
                        load_meta<D>(mnext, C.edge_acc, hoff[k + 1], D, lane);
                    }
                    if (hval[k]) {
#pragma unroll
                        for (int e = 0; e < D; ++e) {
                            const float w = PK ? packed_diff(hr[k][e]) : zr[PK ? 0 : k][e] - ur[PK ? 0 : k][e];
                            atomicAdd(lds_at<unsigned long long>(mcur[e]), to_fixed(w));
                        }
                    }
#pragma unroll
                    for (int e = 0; e < D; ++e) mcur[e] = mnext[e];
                    // many held chunks: one chunk's conversions at a time
                    if constexpr (PK) __builtin_amdgcn_sched_barrier(0);
                }
            }
            if constexpr (!WALK) return;
            Walk cur = walk_at(KR);
            float zc[D], uc[D];
            uint32_t mc[D];
            if (cur.has) walk_load(cur, zc, uc, mc);
            while (cur.has) {
                const Walk nxt = walk_at(cur.k + 1);
                float zn[D], un[D];
                uint32_t mn[D];
                if (nxt.has) walk_load(nxt, zn, un, mn);
                if (lane < cur.cnt) {
#pragma unroll
                    for (int e = 0; e < D; ++e) atomicAdd(lds_at<unsigned long long>(mc[e]), to_fixed(zc[e] - uc[e]));
                }
#pragma unroll
                for (int e = 0; e < D; ++e) {
                    zc[e] = zn[e];
                    uc[e] = un[e];
                    mc[e] = mn[e];
                }
                cur = nxt;
            }
        };
        // B: x_i from its accumulator (less the previous x kept in the high word)
        auto phase_b = [&]() {
            acc_x_update<4, PERSIST>(acc, xprev, C.var_identity ? gam : gmu_row, C.var_identity ? ip.mu_inv : 1.0f, C,
                                     tid, NT);
        };
        // C: check updates (held chunks from registers, walked chunks from memory)
        // residuals per plan wave: rp[j], rd[j] of plan wave wave + j NW
        auto phase_c = [&](float *rp, float *rd) {
            if constexpr (KR > 0) {
                uint32_t mcur[D], mnext[D];
                load_meta<D>(mcur, C.edge_acc, hoff[0], D, lane);
#pragma unroll
                for (int k = 0; k < NH; ++k) {
                    if (k + 1 < NH) load_meta<D>(mnext, C.edge_acc, hoff[k + 1], D, lane);
                    if constexpr (PK) {
                        if (hval[k]) {
                            float zz[D], uu[D];
#pragma unroll
                            for (int e = 0; e < D; ++e) {
                                zz[e] = lo_h2f(hr[k][e]);
                                uu[e] = hi_h2f(hr[k][e]);
                            }
                            check_update<D, 2, true>(zz, uu, mcur, xs, ip.rho, rp[k / KH], rd[k / KH]);
#pragma unroll
                            for (int e = 0; e < D; ++e) hr[k][e] = pack_h2(zz[e], uu[e]);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    } else if (hval[k]) {
                        check_update<D, 2, true>(zr[k], ur[k], mcur, xs, ip.rho, rp[k / KH], rd[k / KH]);
                        if constexpr (!PERSIST) {
#pragma unroll
                            for (int e = 0; e < D; ++e) {
                                const size_t p = hoff[k] + e * kWave + lane;
                                st_state<HALF>(gz, p, zr[k][e]);
                                st_state<HALF>(gu, p, ur[k][e]);
                            }
                        }
                    }
#pragma unroll
                    for (int e = 0; e < D; ++e) mcur[e] = mnext[e];
                }
            }
            if constexpr (!WALK) return;
            Walk cur = walk_at(KR);
            float zc[D], uc[D];
            uint32_t mc[D];
            if (cur.has) walk_load(cur, zc, uc, mc);
            while (cur.has) {
                const Walk nxt = walk_at(cur.k + 1);
                float zn[D], un[D];
                uint32_t mn[D];
                if (nxt.has) walk_load(nxt, zn, un, mn);
                if (lane < cur.cnt) {
                    check_update<D, 2, true>(zc, uc, mc, xs, ip.rho, rp[0], rd[0]);
#pragma unroll
                    for (int e = 0; e < D; ++e) {
                        const size_t p = cur.off + e * kWave + lane;
                        st_state<HALF>(gz, p, zc[e]);
                        st_state<HALF>(gu, p, uc[e]);
                    }
                }
#pragma unroll
                for (int e = 0; e < D; ++e) {
                    zc[e] = zn[e];
                    uc[e] = un[e];
                    mc[e] = mn[e];
                }
                cur = nxt;
            }
        };
        auto publish = [&](int buf, const float *rp, const float *rd) {
#pragma unroll
            for (int j = 0; j < VW; ++j) {
                const int v = wave + j * NW;  // wave-uniform
                const float a = wave_sum(rp[j]), b = wave_sum(rd[j]);
                if (lane == 0 && v < W) {
                    s_red[buf][0][v] = a;
                    s_red[buf][1][v] = b;
                }
            }
        };
        auto converged = [&](int buf) -> bool {  // identical result in every wave
            const float a = lane < W ? s_red[buf][0][lane] : 0.0f;
            const float b = lane < W ? s_red[buf][1][lane] : 0.0f;
            return row0_sum(a) < thr && row0_sum(b) < thr;
        };

        int iters;
        bool conv = false;
        if constexpr (PERSIST) {
            // iteration it = B, C, then the next iteration's A (after a barrier: A adds
            // into the entries C reads x from); the stopping test reads the residuals
            // C published, after the barrier that follows that A
            int it = 1;
            phase_a();
            wg_barrier<true>();
            for (;; ++it) {
                phase_b();
                wg_barrier<true>();
                float rp[VW] = {}, rd[VW] = {};
                phase_c(rp, rd);
                publish(it & 1, rp, rd);
                wg_barrier<true>();
                phase_a();
                wg_barrier<true>();
                if (__builtin_amdgcn_readfirstlane(converged(it & 1))) { conv = true; break; }
                if (it >= ip.max_iter) break;
            }
            iters = conv ? it : ip.max_iter;
            // the last phase A accumulated into the entries holding x: restore the last x
            for (int i = tid; i < C.n; i += NT) acc[i] = (unsigned long long)as_global(xprev)[i] << 32;
            __syncthreads();
        } else {
            const int it = launch + 1;
            phase_a();
            wg_barrier<true>();
            phase_b();
            wg_barrier<true>();
            float rp[VW] = {}, rd[VW] = {};
            phase_c(rp, rd);
            publish(0, rp, rd);
            wg_barrier<true>();
            conv = converged(0);
            iters = it;
            const bool fin = __builtin_amdgcn_readfirstlane(conv || it >= ip.max_iter);
            if (tid == 0) {
                sa.st[f].iter = it;
                if (fin) sa.st[f].done = 1;
                else list_unfinished(f);
            }
            if (!fin) {
                wg_barrier<true>();  // LDS reuse by the next frame of this workgroup
                continue;
            }
        }

        // -- epilogue: x, iteration count and certificate flags ----------------------
        const int64_t xoff = fb.x_off ? uniform_i64(fb.x_off[f]) : (int64_t)f * C.n;
        float frac = 0.0f;
        for (int i = tid; i < C.n; i += NT) {
            const float x = xs[2 * i];
            fb.x_out[xoff + (C.var_identity ? i : C.var_orig[i])] = x;
            frac = fmaxf(frac, fminf(x, 1.0f - x));
        }
        bool odd = false;
        for (int c = wave; c < C.nchunks; c += NW) {
            const ChunkDesc h = chunk_desc(C, c);
            if (lane < h.cnt) {
                bool par = false;
                for (int e = 0; e < D; ++e) par ^= (xs[2 * (C.edge_meta[h.off + e * kWave + lane] & 0xffffu)] >= 0.5f);
                odd |= par;
            }
        }
        // frac > 1e-3 exactly: 1e-3f is the least float above 1e-3
        const bool nonint = frac >= 1e-3f;
        // workgroup votes through the LDS tail (a library vote would bring static LDS)
        const bool wodd = __ballot(odd) != 0ull, wnonint = __ballot(nonint) != 0ull;
        if (lane == 0) {
            s_vote[wave] = wodd;
            s_vote[kMaxWaves + wave] = wnonint;
        }
        __syncthreads();
        if (tid == 0) {
            int any_odd = 0, any_nonint = 0;
            for (int w = 0; w < NW; ++w) {
                any_odd |= s_vote[w];
                any_nonint |= s_vote[kMaxWaves + w];
            }
            uint8_t fl = conv ? 0x01 : 0x00;
            if (!any_nonint) fl |= 0x02;
            if (!any_odd) fl |= 0x04;
            if ((fl & 0x07) == 0x07) fl |= 0x08;
            fb.iters_out[f] = iters;
            fb.flags_out[f] = fl;
            if (fb.done) {
                __threadfence_system();
                __hip_atomic_store(fb.done + f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        // state export in CSR edge order (persistent-global form; the streamed form
        // exports with its own kernel after the last launch)
        if constexpr (PERSIST) {
            if (sio.z_out) {
                const size_t fb0 = (size_t)f * C.E;
#pragma unroll
                for (int k = 0; k < NH; ++k)
#pragma unroll
                    for (int e = 0; e < D; ++e)
                        if (hval[k]) {
                            const int ce = csr_row(C.edge_csr, hoff[k] + e * kWave)[lane];
                            sio.z_out[fb0 + ce] = PK ? lo_h2f(hr[k][e]) : zr[PK ? 0 : k][e];
                            sio.u_out[fb0 + ce] = PK ? hi_h2f(hr[k][e]) : ur[PK ? 0 : k][e];
                        }
                for (int k = KR; k < cpt; ++k) {
                    const int c = wave + k * W;
                    if (c >= C.nchunks) break;
                    const ChunkDesc h = chunk_desc(C, c);
                    if (lane < h.cnt) {
                        for (int e = 0; e < D; ++e) {
                            const size_t p = h.off + e * kWave + lane;
                            const int ce = C.edge_csr[p];
                            sio.z_out[fb0 + ce] = ld_state<HALF>(gz, p);
                            sio.u_out[fb0 + ce] = ld_state<HALF>(gu, p);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Streamed form set-up: zero (or load) each frame's state, flag invalid frames.
template <bool HALF>
__global__ void __launch_bounds__(256)
k_stream_init(const DevCode *__restrict__ codes, FrameBatch fb, StateIO sio, StreamArgs sa, float mu_inv) {
    const int f = blockIdx.x;
    if (f >= fb.nframes) return;
    if (f == 0 && threadIdx.x < 2) sa.active_count[threadIdx.x] = 0;
    // every frame is on the list launch 0 works through (as if launch -1 had made it);
    // launch 0 appends at entry 0
    if (threadIdx.x == 0) sa.alist[(size_t)fb.nframes + f] = f;
    if (f == 0 && threadIdx.x == 0) {
        sa.alist_cnt[2] = fb.nframes;
        sa.alist_cnt[0] = 0;
    }
    const int ci = fb.code_of_frame ? uniform_i32(fb.code_of_frame[f]) : 0;
    const DevCode &C = codes[ci];
    const int64_t loff = fb.llr_off ? uniform_i64(fb.llr_off[f]) : (int64_t)f * C.n;
    const int any_bad = frame_invalid(fb, f);
    const size_t base = (size_t)f * C.E_int;
    for (int p = threadIdx.x; p < C.E_int; p += blockDim.x) {
        float z0 = 0.0f, u0 = 0.0f;
        const int ce = C.edge_csr[p];
        if (sio.z_in && ce >= 0) {
            z0 = sio.z_in[(size_t)f * C.E + ce];
            u0 = sio.u_in[(size_t)f * C.E + ce];
        }
        st_state<HALF>(sa.z, base + p, z0);
        st_state<HALF>(sa.u, base + p, u0);
    }
    if (sa.gmu && !C.var_identity) {
        float *row = sa.gmu + (size_t)f * sa.gmu_stride;
        for (int i = threadIdx.x; i < C.n; i += blockDim.x) row[i] = fb.llr[loff + C.var_orig[i]] * mu_inv;
    }
    if (any_bad) {
        const int64_t xoff = fb.x_off ? uniform_i64(fb.x_off[f]) : (int64_t)f * C.n;
        for (int i = threadIdx.x; i < C.n; i += blockDim.x) fb.x_out[xoff + i] = 0.5f;
    }
    if (threadIdx.x == 0) {
        sa.st[f].iter = 0;
        sa.st[f].done = any_bad ? 1 : 0;
        if (any_bad) {
            fb.iters_out[f] = 0;
            fb.flags_out[f] = 0x80;
        }
    }
}

hipError_t launch_stream_init(const DevCode *codes_dev, int nframes, const LaunchConfig &cfg,
                              const FrameBatch &fb, const StateIO &sio, const StreamArgs &sa,
                              const IterParams &ip, hipStream_t stream) {
    if (nframes <= 0) return hipSuccess;
    if (cfg.half)
        hipLaunchKernelGGL(k_stream_init<true>, dim3(nframes), dim3(256), 0, stream, codes_dev, fb, sio, sa,
                           ip.mu_inv);
    else
        hipLaunchKernelGGL(k_stream_init<false>, dim3(nframes), dim3(256), 0, stream, codes_dev, fb, sio, sa,
                           ip.mu_inv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Instantiation table.

template <int DMIN, int DMAX, int CPT, int VPT, bool RES, bool PERSIST, int SM, bool HALF, int MAXT = kMaxThreads,
          int DV = 0, bool STG = false>
static hipError_t go(const LaunchConfig &cfg, const DevCode *codes, const FrameBatch &fb, const IterParams &ip,
                     const StateIO &sio, const StreamArgs &sa, hipStream_t stream, KernelQuery *q) {
    if (cfg.threads > MAXT) return hipErrorInvalidConfiguration;
    auto kern = k_decode<DMIN, DMAX, CPT, VPT, RES, PERSIST, SM, HALF, MAXT, DV, STG>;
    if (cfg.lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)cfg.lds_bytes);
        if (e != hipSuccess) return e;
    }
    if (q) {
        hipFuncAttributes fa{};
        hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kern));
        if (e != hipSuccess) return e;
        q->vgprs = fa.numRegs;
        q->static_lds = (int)fa.sharedSizeBytes;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&q->occupancy, kern, cfg.threads, cfg.lds_bytes);
    }
    hipLaunchKernelGGL(kern, dim3(cfg.grid), dim3(cfg.threads), cfg.lds_bytes, stream, codes, fb, ip, sio, sa,
                       cfg.lds_E, cfg.slot_stride, cfg.state_stride);
    return hipGetLastError();
}

template <int DMIN, int DMAX>
static hipError_t go_range(const LaunchConfig &cfg, const DevCode *codes, const FrameBatch &fb,
                           const IterParams &ip, const StateIO &sio, const StreamArgs &sa, hipStream_t stream,
                           KernelQuery *q) {
#define LPD_GO(...) return go<DMIN, DMAX, __VA_ARGS__>(cfg, codes, fb, ip, sio, sa, stream, q)
    switch (cfg.form) {
        case Form::Resident:
            // register budget: degree-6 codes only (the host never selects it otherwise)
            if constexpr (DMIN == 6 && DMAX == 6) {
                // one chunk per wave (codes with m <= 1024): fewer registers, more
                // workgroups per CU
                if (cfg.cpt_tmpl == 1 && cfg.vpt_tmpl == 4 && cfg.dv == 3) LPD_GO(1, 4, true, true, 1, false, 768, 3);
                if (cfg.cpt_tmpl == 1 && cfg.vpt_tmpl == 4) LPD_GO(1, 4, true, true, 1, false, 768);
                if (cfg.cpt_tmpl == 2 && cfg.vpt_tmpl == 4 && cfg.dv == 3) LPD_GO(2, 4, true, true, 1, false, 768, 3);
                if (cfg.cpt_tmpl == 2 && cfg.vpt_tmpl == 8 && cfg.dv == 3) LPD_GO(2, 8, true, true, 1, false, 768, 3);
                if (cfg.cpt_tmpl == 2 && cfg.vpt_tmpl == 4) LPD_GO(2, 4, true, true, 1, false, 768);
                if (cfg.cpt_tmpl == 2 && cfg.vpt_tmpl == 8) LPD_GO(2, 8, true, true, 1, false, 768);
                if (cfg.cpt_tmpl == 4 && cfg.dv == 3) LPD_GO(4, 0, true, true, 1, false, 1024, 3);
                if (cfg.cpt_tmpl == 4) LPD_GO(4, 0, true, true, 1, false, 1024);
            }
            // checks of degree 6..8: z, u of up to eight chunks per wave in registers,
            // variables read from the code's tables (VPT 0); the more chunks per
            // wave, the fewer waves (the register file holds the frame either way)
            // checks of degree up to 16, one chunk per wave: z, u of the chunk in registers
            if constexpr (DMIN == 2 && DMAX == kMaxD) {
                if (cfg.cpt_tmpl == 1) LPD_GO(1, 0, true, true, 1, false);
            }
            if constexpr (DMIN == 6 && DMAX == 8) {
                if (cfg.cpt_tmpl == 1) LPD_GO(1, 0, true, true, 1, false);
                if (cfg.cpt_tmpl == 2) LPD_GO(2, 0, true, true, 1, false);
                if (cfg.cpt_tmpl == 4) LPD_GO(4, 0, true, true, 1, false, 768);
                if (cfg.cpt_tmpl == 8) LPD_GO(8, 0, true, true, 1, false, 512);
            }
            break;
        default:
            // degrees 6..8 are built for the resident form only
            if constexpr (!(DMIN == 6 && DMAX == 8)) {
                // checks above degree 8 use the same builds: their per-check arrays spill
                // 11-18 registers at the 128 a lane has here, but a build for 512 threads
                // (167 registers, no spills) ran the (3,13) n = 1057 code 1.37x slower in
                // the persistent-global form at two workgroups per CU instead of three
                switch (cfg.form) {
                    case Form::PersistentGlobal:
                        if (cfg.slot_mode == 1) LPD_GO(0, 0, false, true, 1, false);
                        if (cfg.slot_mode == 2) LPD_GO(0, 0, false, true, 2, false);
                        LPD_GO(0, 0, false, true, 0, false);
                    case Form::Streamed:
                        if (cfg.slot_mode == 1) {
                            // register-held chunks: degree-6 codes only (DMAX = 8 register arrays spill)
                            if constexpr (DMIN == 6 && DMAX == 6) {
                                if (cfg.staged && cfg.cpt_tmpl == 2 && cfg.threads <= 768 && !cfg.half)
                                    LPD_GO(2, 0, false, false, 1, false, 768, 0, true);
                                if (cfg.cpt_tmpl == 2 && cfg.threads <= 768 && !cfg.half) LPD_GO(2, 0, false, false, 1, false, 768);
                                if (cfg.cpt_tmpl == 2 && cfg.threads <= 768 && cfg.half) LPD_GO(2, 0, false, false, 1, true, 768);
                                if (cfg.cpt_tmpl == 2 && !cfg.half) LPD_GO(2, 0, false, false, 1, false);
                                if (cfg.cpt_tmpl == 2 && cfg.half) LPD_GO(2, 0, false, false, 1, true);
                            }
                            if (!cfg.half) LPD_GO(0, 0, false, false, 1, false);
                            LPD_GO(0, 0, false, false, 1, true);
                        }
                        if (cfg.slot_mode == 2) {
                            if (!cfg.half) LPD_GO(0, 0, false, false, 2, false);
                            LPD_GO(0, 0, false, false, 2, true);
                        }
                        if (!cfg.half) LPD_GO(0, 0, false, false, 0, false);
                        LPD_GO(0, 0, false, false, 0, true);
                    default:
                        break;
                }
            }
            break;
    }
#undef LPD_GO
    return hipErrorInvalidValue;
}

// two frames per workgroup (resident form, see k_decode_pair)
static hipError_t go_pair(const LaunchConfig &cfg, const DevCode *codes, const FrameBatch &fb, const IterParams &ip,
                          const StateIO &sio, hipStream_t stream, KernelQuery *q) {
    if (cfg.threads != kPairWaves * kWave || cfg.vpt_tmpl != 4) return hipErrorInvalidConfiguration;
    auto kern = k_decode_pair<4>;
    if (cfg.lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)cfg.lds_bytes);
        if (e != hipSuccess) return e;
    }
    if (q) {
        hipFuncAttributes fa{};
        hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kern));
        if (e != hipSuccess) return e;
        q->vgprs = fa.numRegs;
        q->static_lds = (int)fa.sharedSizeBytes;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&q->occupancy, kern, cfg.threads, cfg.lds_bytes);
    }
    hipLaunchKernelGGL(kern, dim3(cfg.grid), dim3(cfg.threads), cfg.lds_bytes, stream, codes, fb, ip, sio,
                       cfg.pair_host[0], cfg.pair_host[1], cfg.lds_E);
    return hipGetLastError();
}

static int static_lds_bytes(const void *kern) {
    hipFuncAttributes fa{};
    return hipFuncGetAttributes(&fa, kern) == hipSuccess ? (int)fa.sharedSizeBytes : -1;
}

// large check-regular codes with the accumulator exchange (see k_decode_acc)
template <int D, int KR, bool HALF, bool PERSIST, int VW = 1>
static hipError_t go_acc1(const LaunchConfig &cfg, const DevCode *codes, const FrameBatch &fb, const IterParams &ip,
                          const StateIO &sio, const StreamArgs &sa, hipStream_t stream, KernelQuery *q) {
    if (cfg.threads > kMaxThreads / VW) return hipErrorInvalidConfiguration;
    auto kern = k_decode_acc<D, KR, HALF, PERSIST, VW>;
    // the kernel addresses LDS absolutely: its dynamic array must start at address 0
    static const int static_lds = static_lds_bytes(reinterpret_cast<const void *>(kern));
    if (static_lds != 0) return hipErrorInvalidConfiguration;
    // the 8 n bytes of accumulators, then the residual slots and the frame index
    const size_t lds = cfg.lds_bytes + kAccTailBytes;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (q) {
        hipFuncAttributes fa{};
        hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kern));
        if (e != hipSuccess) return e;
        q->vgprs = fa.numRegs;
        q->static_lds = (int)kAccTailBytes;  // the tail plays the part of static LDS
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&q->occupancy, kern, cfg.threads, lds);
    }
    hipLaunchKernelGGL(kern, dim3(cfg.grid), dim3(cfg.threads), lds, stream, codes, fb, ip, sio, sa,
                       cfg.state_stride);
    return hipGetLastError();
}

static hipError_t go_acc(const LaunchConfig &cfg, const DevCode *codes, const FrameBatch &fb, const IterParams &ip,
                         const StateIO &sio, const StreamArgs &sa, hipStream_t stream, KernelQuery *q) {
    const bool pg = cfg.form == Form::PersistentGlobal;
    // held chunks per wave instantiated (see acc_held_chunks in lpdec_host.cpp)
#define LPD_ACC_S(D, KR)                                                                          \
    if (!pg && cfg.acc_d == D && cfg.acc_kr == KR) {                                              \
        if (cfg.half) return go_acc1<D, KR, true, false>(cfg, codes, fb, ip, sio, sa, stream, q); \
        return go_acc1<D, KR, false, false>(cfg, codes, fb, ip, sio, sa, stream, q);              \
    }
#define LPD_ACC_P(D, KR) \
    if (pg && !cfg.half && cfg.acc_d == D && cfg.acc_kr == KR) return go_acc1<D, KR, false, true>(cfg, codes, fb, ip, sio, sa, stream, q);
// acc_kr = 2 kAccAllHeld: every chunk held, two plan waves per hardware wave
#define LPD_ACC_P2(D) \
    if (pg && !cfg.half && cfg.acc_d == D && cfg.acc_kr == 2 * kAccAllHeld) return go_acc1<D, kAccAllHeld, false, true, 2>(cfg, codes, fb, ip, sio, sa, stream, q);
#define LPD_ACC_PH(D, KR) \
    if (pg && cfg.half && cfg.acc_d == D && cfg.acc_kr == KR) return go_acc1<D, KR, true, true>(cfg, codes, fb, ip, sio, sa, stream, q);
    if (cfg.form == Form::Resident) return hipErrorInvalidValue;
    LPD_ACC_S(6, 0)
    LPD_ACC_S(6, 2)
    LPD_ACC_S(8, 0)
    LPD_ACC_S(8, 2)
    LPD_ACC_P(6, 0)
    LPD_ACC_P(6, 1)
    LPD_ACC_P(8, 0)
    LPD_ACC_P(8, 1)
    LPD_ACC_P2(6)
    LPD_ACC_PH(6, 8)
    LPD_ACC_PH(6, 4)
    LPD_ACC_PH(8, 4)
    LPD_ACC_PH(8, 8)
#undef LPD_ACC_S
#undef LPD_ACC_P
#undef LPD_ACC_PH
#undef LPD_ACC_P2
    return hipErrorInvalidValue;
}

hipError_t launch_decode(const LaunchConfig &cfg, const DevCode *codes_dev, const FrameBatch &fb,
                         const IterParams &ip, const StateIO &sio, const StreamArgs &sa, hipStream_t stream) {
    if (cfg.pair) return go_pair(cfg, codes_dev, fb, ip, sio, stream, nullptr);
    if (cfg.acc) return go_acc(cfg, codes_dev, fb, ip, sio, sa, stream, nullptr);
    if (cfg.dclass == 0) return go_range<6, 6>(cfg, codes_dev, fb, ip, sio, sa, stream, nullptr);
    if (cfg.dclass == 2) return go_range<6, 8>(cfg, codes_dev, fb, ip, sio, sa, stream, nullptr);
    if (cfg.dclass == 3) return go_range<2, kMaxD>(cfg, codes_dev, fb, ip, sio, sa, stream, nullptr);
    return go_range<2, 8>(cfg, codes_dev, fb, ip, sio, sa, stream, nullptr);
}

hipError_t decode_query(const LaunchConfig &cfg, KernelQuery *q) {
    FrameBatch fb{};
    IterParams ip{};
    StateIO sio{};
    StreamArgs sa{};
    *q = KernelQuery{};
    if (cfg.pair) return go_pair(cfg, nullptr, fb, ip, sio, nullptr, q);
    if (cfg.acc) return go_acc(cfg, nullptr, fb, ip, sio, sa, nullptr, q);
    if (cfg.dclass == 0) return go_range<6, 6>(cfg, nullptr, fb, ip, sio, sa, nullptr, q);
    if (cfg.dclass == 2) return go_range<6, 8>(cfg, nullptr, fb, ip, sio, sa, nullptr, q);
    if (cfg.dclass == 3) return go_range<2, kMaxD>(cfg, nullptr, fb, ip, sio, sa, nullptr, q);
    return go_range<2, 8>(cfg, nullptr, fb, ip, sio, sa, nullptr, q);
}

// Streamed form: copy the final lane-minor state back to CSR edge order.
template <bool HALF>
__global__ void __launch_bounds__(256)
k_stream_export(const DevCode *__restrict__ codes, int nframes, StateIO sio, StreamArgs sa) {
    const int f = blockIdx.y;
    const DevCode &C = codes[0];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nframes || p >= C.E_int) return;
    const int ce = C.edge_csr[p];
    if (ce < 0) return;
    const size_t src = (size_t)f * C.E_int + p, dst = (size_t)f * C.E + ce;
    sio.z_out[dst] = ld_state<HALF>(sa.z, src);
    sio.u_out[dst] = ld_state<HALF>(sa.u, src);
}

hipError_t launch_stream_export(const DevCode *codes_dev, int nframes, int E_int, bool half, const StateIO &sio,
                                const StreamArgs &sa, hipStream_t stream) {
    if (nframes <= 0) return hipSuccess;
    const dim3 grid((E_int + 255) / 256, nframes);
    if (half) hipLaunchKernelGGL(k_stream_export<true>, grid, dim3(256), 0, stream, codes_dev, nframes, sio, sa);
    else hipLaunchKernelGGL(k_stream_export<false>, grid, dim3(256), 0, stream, codes_dev, nframes, sio, sa);
    return hipGetLastError();
}

}  // namespace lpdec
