// HIP kernels (gfx950) beside the ADMM decoder: the dual subgradient ascent of
// Appendix A and the per-frame bookkeeping behind the ML lower bound of Sec. 5.1.
//
// Paper: Barman, Liu, Draper, Recht, "Decomposition Methods for Large Scale LP
// Decoding" (arXiv 1204.0556).
//
// Both kernels use the code layout of the decoder: checks grouped by degree in
// 64-check chunks with lane-minor edge metadata (slot << 16 | internal
// variable), variables renumbered, var_orig mapping back to the caller's order.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lpdec_aux.h"

namespace lpdec {

namespace {

__device__ __forceinline__ bool finite_f(float a) { return (__float_as_uint(a) & 0x7f800000u) != 0x7f800000u; }

template <int DMIN, int DMAX, typename F>
__device__ __forceinline__ void for_degree(int d, F &&f) {
    if constexpr (DMIN == DMAX) {
        f(std::integral_constant<int, DMIN>{});
    } else {
        if (d == DMIN) f(std::integral_constant<int, DMIN>{});
        else for_degree<DMIN + 1, DMAX>(d, f);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Dual subgradient ascent (Appendix A).  With lambda_e = mu K_e (K an integer
// count: every update adds mu times -1, 0 or +1), one iteration is
//   x_i = [ -gamma_i - mu S_i > 0 ],  S_i = sum of K over the variable's edges
//   z_j = argmax over PP_d of K_j^T z  (Algorithm 3; the sign and order of
//         lambda_j are those of K_j because mu > 0)
//   K_e += x_i(e) - z_e
// The x decision is taken in FP64, exactly as the expression reads (no fused
// multiply-add), so it matches an FP64 reference bit for bit; everything else
// is integer.  S_i lives in LDS and is updated with integer atomics (order
// free); K stays in registers, CPT chunks per wave.  The frame stops once no
// K moves (then P_j x = z_j for every check: x is an LP optimum and a
// codeword) or after max_iter iterations.
//
// LDS: S [n] int32, -gamma [n] float, x [n] bytes.
template <int DMIN, int DMAX, int CPT>
__global__ void __launch_bounds__(kMaxThreads)
k_dual(const DevCode *__restrict__ codes, FrameBatch fb, double mu, int max_iter) {
    extern __shared__ __attribute__((aligned(16))) int dlds[];
    __shared__ int s_frame;
    const DevCode &C = codes[0];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), NT = blockDim.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    int *S = dlds;
    float *ng = reinterpret_cast<float *>(dlds + C.n);
    uint8_t *xb = reinterpret_cast<uint8_t *>(dlds + 2 * C.n);

    // this lane's checks: chunk c = wave + k * waves; their edge metadata is held
    // in registers when it fits (up to 32 entries per lane), else re-read from the
    // (cache-resident) code table
    constexpr bool MREG = CPT * DMAX <= 32;
    int cdeg[CPT];
    const __attribute__((address_space(1))) uint32_t *cmeta[CPT];
    uint32_t cm[MREG ? CPT : 1][MREG ? DMAX : 1];
    bool cval[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int c = wave + k * C.waves;
        const bool has = (wave < C.waves) && (k < C.cpt) && (c < C.nchunks);
        cdeg[k] = has ? __builtin_amdgcn_readfirstlane(as_global(C.chunk_deg)[c]) : 0;
        cmeta[k] = as_global(C.edge_meta) + (has ? __builtin_amdgcn_readfirstlane(as_global(C.chunk_off)[c]) : 0) + lane;
        cval[k] = has && (lane < as_global(C.chunk_cnt)[c]);
        if constexpr (MREG) {
#pragma unroll
            for (int e = 0; e < DMAX; ++e) cm[k][e] = (cval[k] && e < cdeg[k]) ? cmeta[k][e * kWave] : 0u;
        }
    }

    // Workgroup-uniform values (the frame index, the outcome of a workgroup
    // vote) are moved to scalar registers with readfirstlane, so that every
    // branch on them is uniform: the frame loop then has one shape for all
    // lanes, and lane 0's fetch of the next frame is never separated from the
    // lanes waiting for it.
    for (;;) {
        if (tid == 0) s_frame = atomicAdd(fb.queue, 1);
        __syncthreads();
        const int f = __builtin_amdgcn_readfirstlane(s_frame);
        __syncthreads();
        if (f >= fb.nframes) break;
        const float *gam = fb.llr + (size_t)f * C.n;
        float *xo = fb.x_out + (size_t)f * C.n;
        bool bad = false;
        for (int i = tid; i < C.n; i += NT) {
            const float g = gam[C.var_identity ? i : C.var_orig[i]];
            bad |= !finite_f(g);
            ng[i] = -g;
            S[i] = 0;
        }
        const int frame_bad = __builtin_amdgcn_readfirstlane(__syncthreads_or(bad));
        if (frame_bad) {
            for (int i = tid; i < C.n; i += NT) xo[i] = 0.5f;
            if (tid == 0) {
                fb.iters_out[f] = 0;
                fb.flags_out[f] = 0x80;
            }
        } else {
            int K[CPT][DMAX];
#pragma unroll
            for (int k = 0; k < CPT; ++k)
#pragma unroll
                for (int e = 0; e < DMAX; ++e) K[k][e] = 0;

            int it = 0;
            bool conv = false;
            while (it < max_iter) {
                ++it;
                // x-update: the sign of the reduced cost, in FP64
                for (int i = tid; i < C.n; i += NT) {
                    const double t = (double)ng[i] - mu * (double)S[i];
                    xb[i] = t > 0.0 ? 1 : 0;
                }
                __syncthreads();
                // z-update (Algorithm 3) and multiplier step, check by check
                bool moved = false;
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (!cval[k]) continue;
                    for_degree<DMIN, DMAX>(cdeg[k], [&](auto dc) {
                        constexpr int D = decltype(dc)::value;
                        // r = #positive entries; i_p = first smallest positive entry,
                        // i_n = first largest non-positive entry
                        int r = 0, ip = -1, in = -1;
                        int kp = 0x7fffffff, kn = -0x7fffffff - 1;
#pragma unroll
                        for (int e = 0; e < D; ++e) {
                            const int v = K[k][e];
                            if (v > 0) {
                                ++r;
                                if (v < kp) { kp = v; ip = e; }
                            } else if (v > kn) {
                                kn = v;
                                in = e;
                            }
                        }
                        // odd r: add i_n when that gains more than dropping i_p loses
                        const bool odd = r & 1;
                        const bool add_n = odd && in >= 0 && (long long)kp + (long long)kn > 0;
#pragma unroll
                        for (int e = 0; e < D; ++e) {
                            int z = K[k][e] > 0 ? 1 : 0;
                            if (odd && e == ip && !add_n) z = 0;
                            if (add_n && e == in) z = 1;
                            const int var = (int)((MREG ? cm[k][MREG ? e : 0] : cmeta[k][e * kWave]) & 0xffffu);
                            const int delta = (int)xb[var] - z;
                            if (delta != 0) {
                                K[k][e] += delta;
                                atomicAdd(S + var, delta);
                                moved = true;
                            }
                        }
                    });
                }
                if (!__builtin_amdgcn_readfirstlane(__syncthreads_or(moved))) {
                    conv = true;
                    break;
                }
            }
            // epilogue: x (the last x-update), iterations, flags
            bool odd = false;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                if (!cval[k]) continue;
                bool par = false;
#pragma unroll
                for (int e = 0; e < DMAX; ++e)
                    if (e < cdeg[k]) par ^= xb[cmeta[k][e * kWave] & 0xffffu] != 0;
                odd |= par;
            }
            for (int i = tid; i < C.n; i += NT) xo[C.var_identity ? i : C.var_orig[i]] = (float)xb[i];
            const int any_odd = __syncthreads_or(odd);
            if (tid == 0) {
                uint8_t fl = 0x02 | (conv ? 0x01 : 0x00);
                if (!any_odd) fl |= 0x04;
                if ((fl & 0x07) == 0x07) fl |= 0x08;
                fb.iters_out[f] = conv ? it : max_iter;
                fb.flags_out[f] = fl;
            }
        }
        __syncthreads();  // LDS reuse by the next frame
    }
}

template <int DMIN, int DMAX, int CPT>
static hipError_t go_dual(const DualLaunch &L, const DevCode *codes, const FrameBatch &fb, double mu, int max_iter,
                          hipStream_t stream, int *occ) {
    auto kern = k_dual<DMIN, DMAX, CPT>;
    if (L.lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes);
        if (e != hipSuccess) return e;
    }
    if (occ) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, L.threads, L.lds_bytes);
    hipLaunchKernelGGL(kern, dim3(L.grid), dim3(L.threads), L.lds_bytes, stream, codes, fb, mu, max_iter);
    return hipGetLastError();
}

template <int DMIN, int DMAX>
static hipError_t go_dual_cpt(const DualLaunch &L, const DevCode *codes, const FrameBatch &fb, double mu,
                              int max_iter, hipStream_t stream, int *occ) {
    if (L.cpt <= 2) return go_dual<DMIN, DMAX, 2>(L, codes, fb, mu, max_iter, stream, occ);
    if (L.cpt <= 4) return go_dual<DMIN, DMAX, 4>(L, codes, fb, mu, max_iter, stream, occ);
    if (L.cpt <= 8) return go_dual<DMIN, DMAX, 8>(L, codes, fb, mu, max_iter, stream, occ);
    return hipErrorInvalidValue;
}

hipError_t launch_dual(const DualLaunch &L, const DevCode *codes, const FrameBatch &fb, double mu, int max_iter,
                       hipStream_t stream, int *occ) {
    if (L.dclass == 0) return go_dual_cpt<6, 6>(L, codes, fb, mu, max_iter, stream, occ);
    return go_dual_cpt<2, 8>(L, codes, fb, mu, max_iter, stream, occ);
}

// ---------------------------------------------------------------------------
// ML lower-bound bookkeeping (Sec. 5.1), one workgroup per frame.  xhat_i =
// [x_i >= 1/2]; bit errors against the transmitted word (all-zero when `sent`
// is null); costs gamma^T xhat and gamma^T sent summed in FP64; the codeword
// test H xhat = 0 is recomputed from the code.  outcome: bit0 word error, bit1
// xhat is a codeword, bit2 an ML decoder errs too (word error, codeword, and
// gamma^T xhat < gamma^T sent).
__device__ __forceinline__ double wave_sum_f64(double a) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
    return a;
}
__device__ __forceinline__ int wave_sum_i32(int a) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
    return a;
}

__global__ void __launch_bounds__(256) k_evaluate(const DevCode *__restrict__ codes, EvalBatch eb) {
    extern __shared__ __attribute__((aligned(16))) uint8_t xh[];  // xhat in internal variable order
    __shared__ double s_c[2][4];
    __shared__ int s_b[4];
    const int f = blockIdx.x;
    if (f >= eb.nframes) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const DevCode &C = codes[eb.code_of_frame ? eb.code_of_frame[f] : 0];
    const int64_t lo = eb.llr_off ? eb.llr_off[f] : (int64_t)f * C.n;
    const int64_t xo = eb.x_off ? eb.x_off[f] : (int64_t)f * C.n;
    double ch = 0.0, cs = 0.0;
    int be = 0;
    for (int i = tid; i < C.n; i += blockDim.x) {
        const int oi = C.var_identity ? i : C.var_orig[i];
        const bool h = eb.x[xo + oi] >= 0.5f;
        const bool s = eb.sent ? eb.sent[xo + oi] != 0 : false;
        const double g = (double)eb.llr[lo + oi];
        xh[i] = h ? 1 : 0;
        be += h != s;
        if (h) ch += g;
        if (s) cs += g;
    }
    ch = wave_sum_f64(ch);
    cs = wave_sum_f64(cs);
    be = wave_sum_i32(be);
    if (lane == 0) {
        s_c[0][wave] = ch;
        s_c[1][wave] = cs;
        s_b[wave] = be;
    }
    __syncthreads();
    bool odd = false;
    for (int c = wave; c < C.nchunks; c += 4) {
        const int d = C.chunk_deg[c], off = C.chunk_off[c];
        if (lane < C.chunk_cnt[c]) {
            bool par = false;
            for (int e = 0; e < d; ++e) par ^= xh[C.edge_meta[off + e * kWave + lane] & 0xffffu] != 0;
            odd |= par;
        }
    }
    const int any_odd = __syncthreads_or(odd);
    if (tid == 0) {
        const double th = (s_c[0][0] + s_c[0][1]) + (s_c[0][2] + s_c[0][3]);
        const double ts = (s_c[1][0] + s_c[1][1]) + (s_c[1][2] + s_c[1][3]);
        const int tb = (s_b[0] + s_b[1]) + (s_b[2] + s_b[3]);
        uint8_t o = 0;
        if (tb) o |= 0x01;
        if (!any_odd) o |= 0x02;
        if (tb && !any_odd && th < ts) o |= 0x04;
        eb.bit_errors[f] = tb;
        eb.cost_hat[f] = th;
        eb.cost_sent[f] = ts;
        eb.outcome[f] = o;
    }
}

// ---------------------------------------------------------------------------
// Input check before a decode: flags_out[f] = 0x80 when frame f holds a
// non-finite LLR (tested on the bit pattern), else 0.  The decoder kernels are
// built without NaN semantics and take their invalid-frame decision from here.
__global__ void __launch_bounds__(256) k_check_finite(const DevCode *__restrict__ codes, FrameBatch fb) {
    const int f = blockIdx.x;
    if (f >= fb.nframes) return;
    const DevCode &C = codes[fb.code_of_frame ? fb.code_of_frame[f] : 0];
    const int64_t lo = fb.llr_off ? fb.llr_off[f] : (int64_t)f * C.n;
    bool bad = false;
    for (int i = threadIdx.x; i < C.n; i += blockDim.x) bad |= !finite_f(fb.llr[lo + i]);
    const int any = __syncthreads_or(bad);
    if (threadIdx.x == 0) fb.flags_out[f] = any ? 0x80 : 0;
}

hipError_t launch_check_finite(const DevCode *codes, const FrameBatch &fb, hipStream_t stream) {
    if (fb.nframes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_finite, dim3(fb.nframes), dim3(256), 0, stream, codes, fb);
    return hipGetLastError();
}

hipError_t launch_evaluate(const DevCode *codes, const EvalBatch &eb, int nmax, hipStream_t stream) {
    if (eb.nframes <= 0) return hipSuccess;
    const size_t lds = ((size_t)nmax + 15) / 16 * 16;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_evaluate),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_evaluate, dim3(eb.nframes), dim3(256), lds, stream, codes, eb);
    return hipGetLastError();
}

}  // namespace lpdec
