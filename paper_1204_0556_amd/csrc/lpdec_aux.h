// Launch interface of the auxiliary kernels (lpdec_aux.hip): the dual
// subgradient ascent of Appendix A and the ML lower-bound bookkeeping of
// Sec. 5.1.  Not part of the ABI.
#pragma once

#include "lpdec_internal.h"

namespace lpdec {

struct DualLaunch {
    int dclass;        // 0: every check has degree 6; 1: degrees 2..8
    int cpt;           // chunks per wave of the code (<= 8)
    int threads;       // workgroup size (code waves x 64)
    int grid;          // persistent workgroups
    size_t lds_bytes;  // 9 n bytes, rounded up
};

// occ != nullptr: report workgroups per CU instead of launching
hipError_t launch_dual(const DualLaunch &L, const DevCode *codes, const FrameBatch &fb, double mu, int max_iter,
                       hipStream_t stream, int *occ);

struct EvalBatch {
    int nframes;
    const int32_t *code_of_frame;  // device, or null (every frame uses codes[0])
    const int64_t *llr_off;        // device, or null (f * n)
    const int64_t *x_off;          // device, or null (f * n); also indexes `sent`
    const float *llr;
    const float *x;
    const uint8_t *sent;           // transmitted bits, or null (all-zero codeword)
    int32_t *bit_errors;
    double *cost_hat, *cost_sent;
    uint8_t *outcome;
};

hipError_t launch_evaluate(const DevCode *codes, const EvalBatch &eb, int nmax, hipStream_t stream);

// flags_out[f] = 0x80 for frames with a non-finite LLR, else 0 (run before a decode)
hipError_t launch_check_finite(const DevCode *codes, const FrameBatch &fb, hipStream_t stream);

}  // namespace lpdec
