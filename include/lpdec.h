/*
 * lpdec.h -- C ABI of the MI355X (gfx950) ADMM LP decoder.
 *
 * Method: Barman, Liu, Draper, Recht, "Decomposition Methods for Large Scale LP
 * Decoding" (arXiv 1204.0556).  The library solves Feldman's LP relaxation
 *     minimise gamma^T x  s.t.  P_j x in PP_d for every check j    (eq. feldmanLP)
 * with the ADMM iteration of Algorithm 1 (Sec. 3.3), over-relaxed as in Sec. 5.2,
 * each z-update being a Euclidean projection onto the parity polytope PP_d
 * computed from the two-slice characterisation (Sec. 4, Algorithm 2).
 *
 * Conventions for every entry point
 *   - Return value: LPDEC_OK (0) or a negative lpdec_status; a thread-local
 *     message for the last failure is available from lpdec_last_error().
 *   - "host" pointers are read during the call only and stay owned by the caller.
 *   - "device" pointers are HIP device allocations owned by the caller (e.g. torch
 *     tensors); they must stay valid until the work queued on `stream` completes.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Decode
 *     calls are asynchronous on it: outputs are ready when the stream is.  Two
 *     exceptions block the calling thread: the streamed form (one launch per
 *     iteration) queues its launches in blocks of 16, reads after each block how
 *     many frames are still unfinished (so a decode that converges early stops
 *     issuing launches) and returns only after its iterations have run; and a call
 *     with scattered frames (lpdec_decode_multi) first waits for the previous such
 *     call on the same code to finish, because it reuses that call's pinned staging
 *     of the per-frame metadata.
 *   - Arguments are validated on the host before anything is queued; a rejected
 *     call queues no work.  Per-frame problems (non-finite LLRs) are reported in
 *     the frame's flags and never abort the batch.
 */
#ifndef LPDEC_H
#define LPDEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest check degree d = |N_c(j)| the kernels support (Sec. 2: the paper's
 * codes use d = 6 and d = 13).  Codes with a check of degree above 8 decode in
 * the persistent-global and streamed forms, in RESIDENT only with one chunk of
 * checks per wave (at most 1024 checks), and not in the dual decoder. */
#define LPDEC_MAX_CHECK_DEGREE 16

typedef enum {
    LPDEC_OK = 0,
    LPDEC_EINVAL = -1,       /* malformed argument (message says which)            */
    LPDEC_ENOMEM = -2,       /* a device or host allocation failed                 */
    LPDEC_EDEVICE = -3,      /* a HIP runtime call failed                          */
    LPDEC_EUNSUPPORTED = -4, /* valid input outside the supported envelope         */
    LPDEC_EBUSY = -5         /* resource in use (serving queue full)               */
} lpdec_status;

/* Per-frame flag bits written to flags_out. */
#define LPDEC_FLAG_CONVERGED 0x01u /* both residuals fell below tol (Alg. 1 UNTIL)     */
#define LPDEC_FLAG_INTEGRAL 0x02u  /* max_i min(x_i, 1 - x_i) <= 1e-3                   */
#define LPDEC_FLAG_CODEWORD 0x04u  /* H xhat = 0 (mod 2), xhat_i = [x_i >= 1/2]         */
#define LPDEC_FLAG_CERTIFIED 0x08u /* converged, integral and a codeword: the LP optimum
                                      is integral, hence the ML codeword (Sec. 1)       */
#define LPDEC_FLAG_INVALID 0x80u   /* a non-finite LLR: frame not decoded, x = 1/2      */

/* Message storage precision of the state kept between iterations (HBM in the
 * streamed form; registers and per-workgroup scratch in the persistent-global
 * form).  With FP16 every update rounds z and u to FP16 (nearest even) and all
 * arithmetic is FP32; the streamed and persistent-global forms then give bitwise
 * the same results. */
#define LPDEC_STORAGE_FP32 0
#define LPDEC_STORAGE_FP16 1 /* z and u = lambda/mu stored as FP16, FP32 compute     */

/* Execution form. */
#define LPDEC_MODE_AUTO 0     /* fastest form that fits the code                       */
#define LPDEC_MODE_RESIDENT 1 /* one persistent launch; a workgroup keeps a frame's
                                 replicas and duals in registers until it converges
                                 (codes whose checks all have degree 6, or all degrees
                                 6..8, and whose state fits, and codes with a check
                                 above degree 8 that need one chunk of 64 checks per
                                 wave, m <= 1024; see resident_capable)               */
#define LPDEC_MODE_STREAMED 2 /* replicas and duals live in HBM; one launch per
                                 iteration over all unfinished frames                  */
#define LPDEC_MODE_PERSISTENT_GLOBAL 3 /* one persistent launch; per-workgroup state in
                                 global memory (codes too large for registers)         */

typedef struct lpdec_code lpdec_code; /* opaque; holds the device copy of H */

typedef struct {
    float mu;         /* ADMM penalty, > 0 (the paper uses 3, Sec. 5.1)                  */
    float rho;        /* over-relaxation, 1 <= rho < 2 (the paper uses 1.9, Sec. 5.2);
                         rho = 1 is Algorithm 1 exactly                                   */
    int32_t max_iter; /* >= 1 (t_max; 1000 in Sec. 5.1)                                   */
    float tol;        /* epsilon >= 0 (1e-5 in Sec. 5.1); 0 disables the stopping test   */
    int32_t storage;  /* LPDEC_STORAGE_*; FP16 applies to the STREAMED form and to the
                         PERSISTENT_GLOBAL form of one code whose checks all have degree
                         6 or 8 and whose n is too large for LDS slots (the accumulator
                         exchange); AUTO with FP16 picks the latter where it exists, else
                         the former; RESIDENT with FP16: LPDEC_EUNSUPPORTED             */
    int32_t mode;     /* LPDEC_MODE_*                                                     */
} lpdec_params;

/* Paper defaults: mu = 3, rho = 1.9, max_iter = 1000, tol = 1e-5, FP32, AUTO. */
lpdec_params lpdec_default_params(void);

/* Build a decoder for the code with parity-check matrix H (Sec. 2).
 *   m, n      number of checks (rows) and variables (columns), both >= 1
 *   nnz       number of ones in H (edges of the Tanner graph)
 *   row_ptr   host [m+1], CSR row pointers, row_ptr[0] = 0, row_ptr[m] = nnz
 *   col_idx   host [nnz], column indices, strictly increasing within a row
 * Every column must appear in some row (x_i is an average over |N_v(i)| > 0
 * replicas, Sec. 3.2) and every row must have degree 2..LPDEC_MAX_CHECK_DEGREE.
 * The matrix is copied to the device; the caller keeps ownership of its arrays.
 * Errors: LPDEC_EINVAL (malformed CSR, empty column, duplicate index, row of
 * degree < 2), LPDEC_EUNSUPPORTED (degree above the maximum), LPDEC_ENOMEM,
 * LPDEC_EDEVICE.  On error *out is set to NULL. */
lpdec_status lpdec_code_create(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                               const int32_t *col_idx, lpdec_code **out);

/* Release a code and its cached workspaces; waits for work queued on it.  NULL-safe. */
void lpdec_code_destroy(lpdec_code *code);

typedef struct {
    int32_t m, n;
    int64_t nnz;
    int32_t min_check_degree, max_check_degree;
    int32_t resident_capable; /* 1 if LPDEC_MODE_RESIDENT fits this code               */
    int32_t threads_per_frame;/* workgroup size the decode kernels use for this code     */
} lpdec_code_info;

lpdec_status lpdec_code_get_info(const lpdec_code *code, lpdec_code_info *info);

/* Decode `batch` independent frames (Algorithm 1).
 *   llr       device [batch*n] FP32, row-major; gamma_i = log W(y_i|0)/W(y_i|1)
 *             (Sec. 2), e.g. 2 y_i / sigma^2 for BPSK (0 -> +1) over AWGN
 *   p         host; NULL means lpdec_default_params()
 *   x_out     device [batch*n] FP32: the final x in [0,1]^n (the x of the last
 *             iteration run)
 *   iters_out device [batch] int32: iterations run (max_iter if not converged, 0 if invalid)
 *   flags_out device [batch] uint8: LPDEC_FLAG_* bits
 * batch = 0 is a no-op.  The call is asynchronous on `stream`.  Errors:
 * LPDEC_EINVAL (bad parameters or NULL pointers), LPDEC_EUNSUPPORTED (mode not
 * available for this code), LPDEC_ENOMEM (workspace), LPDEC_EDEVICE. */
lpdec_status lpdec_decode(const lpdec_code *code, int32_t batch, const float *llr,
                          const lpdec_params *p, float *x_out, int32_t *iters_out,
                          uint8_t *flags_out, void *stream);

/* lpdec_decode with access to the ADMM state, for checkpoint/resume and for
 * comparing messages after a fixed number of iterations.
 *   z_state, u_state  device [batch*nnz] FP32 in the CSR edge order of H: the
 *             replicas z_j and scaled duals u_j = lambda_j / mu (Sec. 3.4).  Either
 *             both NULL or both given.
 *   state_flags  bit0 LPDEC_STATE_IN: start from the given state instead of zero;
 *                bit1 LPDEC_STATE_OUT: write the final state back.
 * Resuming a run for K2 iterations from the state after K1 reproduces K1+K2
 * iterations exactly when stopping is disabled (tol = 0). */
#define LPDEC_STATE_IN 0x1
#define LPDEC_STATE_OUT 0x2
lpdec_status lpdec_decode_state(const lpdec_code *code, int32_t batch, const float *llr,
                                const lpdec_params *p, float *x_out, int32_t *iters_out,
                                uint8_t *flags_out, float *z_state, float *u_state,
                                int32_t state_flags, void *stream);

/* lpdec_decode for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The call
 * makes no device or host allocation of its own (no hipMalloc, hipFree,
 * hipHostMalloc, event creation or workspace growth): its scratch -- the
 * persistent launch's queue counter and the per-workgroup buffers of the
 * persistent forms -- lives in one static device array of
 * LPDEC_NOALLOC_SCRATCH_BYTES per GPU, loaded with the library and held until
 * the process ends.  The caller still passes llr, x_out, iters_out and flags_out
 * (device, as lpdec_decode).
 *   - Forms: the persistent ones (mode AUTO, RESIDENT or PERSISTENT_GLOBAL, FP32
 *     storage).  The streamed form keeps every frame's state in HBM, which the
 *     array does not hold, and FP16 storage is not offered here: both give
 *     LPDEC_EUNSUPPORTED.
 *   - Size: when the persistent-global form needs per-workgroup buffers, the
 *     grid is cut to what the array holds (results do not depend on the grid);
 *     a code whose single workgroup needs more than the array is rejected with
 *     LPDEC_EUNSUPPORTED (no code within this library's limits does).
 *   - Results are bitwise those of lpdec_decode with the same parameters.
 *   - Every call on one GPU shares that GPU's array, and the array keeps the last
 *     call's contents (each call resets what must start at zero with a kernel,
 *     not a memset).  Calls that overlap on one GPU -- on different streams, or
 *     from different threads -- race on the array and give undefined results:
 *     serialise them.  Asynchronous on `stream`, like lpdec_decode. */
#define LPDEC_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
lpdec_status lpdec_decode_noalloc(const lpdec_code *code, int32_t batch, const float *llr,
                                  const lpdec_params *p, float *x_out, int32_t *iters_out,
                                  uint8_t *flags_out, void *stream);

/* Batched uneven decoding: `nframes` frames drawn from `ncodes` codes, decoded in
 * one persistent launch with per-frame early termination.
 *   codes          host [ncodes] code handles
 *   code_of_frame  host [nframes], values in [0, ncodes)
 *   llr_offset     host [nframes] int64: frame f's LLRs are llr[llr_offset[f] ...
 *                  + n(code) - 1] in the device array `llr`
 *   x_offset       host [nframes] int64: frame f's x goes to x_out[x_offset[f] ...]
 *   iters_out, flags_out  device [nframes]
 * Offsets are checked against llr_len / x_len (elements).  A frame's result does
 * not depend on the other frames of the batch.  When the codes differ in size,
 * the launch hands out frames of larger codes first (processing order only).
 * AUTO picks the register-resident form when every code's checks have degree 6
 * (or all lie in 6..8, or the codes need one chunk per wave) and the largest code
 * fits its register and LDS budget, else the persistent-global form.  FP16 storage and the streamed form are not
 * available here (LPDEC_EUNSUPPORTED). */
lpdec_status lpdec_decode_multi(const lpdec_code *const *codes, int32_t ncodes, int32_t nframes,
                                const int32_t *code_of_frame, const int64_t *llr_offset,
                                const float *llr, int64_t llr_len, const lpdec_params *p,
                                float *x_out, const int64_t *x_offset, int64_t x_len,
                                int32_t *iters_out, uint8_t *flags_out, void *stream);

/* ------------------------------------------------------------------------- */
/* Dual subgradient ascent (Appendix A): the other decomposition the paper
 * describes.  With the un-augmented Lagrangian, x_i = [-gamma_i - sum of the
 * variable's multipliers > 0], each z_j maximises lambda_j^T z over PP_d
 * (Algorithm 3, O(d)), and lambda_j += mu (P_j x - z_j) with constant step mu.
 * Every multiplier is mu times an integer, so the iteration runs on integer
 * counts; the x decision is taken in FP64.  A frame stops when P_j x = z_j for
 * every check (lambda stops moving; x is then an LP optimum and a codeword:
 * converged, integral, codeword and certified are all set) or after max_iter
 * iterations.  x_out holds the last x (0 or 1 per bit).
 *   p  host; uses mu (step size, > 0) and max_iter; NULL = defaults
 * Other arguments as lpdec_decode.  LPDEC_EUNSUPPORTED when the code needs more
 * than 8 check chunks per wave (m > 8192), has a check of degree above 8, or 9 n
 * bytes exceed the LDS. */
lpdec_status lpdec_decode_dual(const lpdec_code *code, int32_t batch, const float *llr,
                               const lpdec_params *p, float *x_out, int32_t *iters_out,
                               uint8_t *flags_out, void *stream);

/* ML lower-bound bookkeeping (Sec. 5.1).  For each frame the estimate is
 * rounded, xhat_i = [x_i >= 1/2], and compared with the transmitted word:
 *   sent        device [batch*n] bytes (nonzero = 1), or NULL for the all-zero
 *               codeword; indexed like x
 *   bit_errors  device [batch] int32: |{i : xhat_i != sent_i}|
 *   cost_hat    device [batch] FP64: gamma^T xhat
 *   cost_sent   device [batch] FP64: gamma^T sent
 *   outcome     device [batch] uint8: LPDEC_EVAL_* bits
 * H xhat = 0 is recomputed from the code.  A word error whose estimate is a
 * codeword cheaper than the transmitted one (gamma is the negative
 * log-likelihood ratio, Sec. 2) would also be an ML decoding error; counting
 * those frames gives a lower bound on the ML word-error rate.  A cost tie counts
 * as an ML success.  Costs are summed in FP64 in a tree order. */
#define LPDEC_EVAL_WORD_ERROR 0x01u
#define LPDEC_EVAL_CODEWORD 0x02u
#define LPDEC_EVAL_ML_ERROR 0x04u
lpdec_status lpdec_evaluate(const lpdec_code *code, int32_t batch, const float *llr, const float *x,
                            const uint8_t *sent, int32_t *bit_errors, double *cost_hat,
                            double *cost_sent, uint8_t *outcome, void *stream);

/* lpdec_evaluate over frames of several codes, laid out as for lpdec_decode_multi
 * (host code_of_frame / llr_offset / x_offset, checked against llr_len / x_len;
 * `sent` is indexed by x_offset). */
lpdec_status lpdec_evaluate_multi(const lpdec_code *const *codes, int32_t ncodes, int32_t nframes,
                                  const int32_t *code_of_frame, const int64_t *llr_offset,
                                  const float *llr, int64_t llr_len, const float *x,
                                  const int64_t *x_offset, int64_t x_len, const uint8_t *sent,
                                  int32_t *bit_errors, double *cost_hat, double *cost_sent,
                                  uint8_t *outcome, void *stream);

/* ------------------------------------------------------------------------- */
/* Launch shape and tuning.  Frames are independent and every sum inside a
 * frame has a fixed order, so the launch shape changes speed only: results are
 * bitwise the same for any workgroups-per-CU setting. */

typedef struct {
    int32_t mode;                  /* the form these figures describe (LPDEC_MODE_*)      */
    int32_t threads;               /* workgroup size = threads per frame                  */
    int32_t lds_bytes;             /* dynamic LDS per workgroup                           */
    int32_t vgprs;                 /* vector registers per lane of the selected kernel    */
    int32_t runtime_blocks_per_cu; /* the HIP runtime's occupancy estimate                */
    int32_t resource_blocks_per_cu;/* workgroups per CU that registers and LDS allow      */
    int32_t blocks_per_cu;         /* what decode launches of this code use now           */
    int32_t variant;               /* streamed form: 0 z,u re-read from HBM in each phase;
                                      1 two chunks per wave in registers, two workgroups
                                      per CU; 2 as 1 with one workgroup per CU staging the
                                      next frame in LDS (direct-to-LDS loads).
                                      resident form, for one code whose checks all have
                                      degree 6 and variables degree 3, planned with two
                                      chunks per wave: 0 one frame per workgroup; 1 two
                                      frames per 12-wave workgroup, placed so that the
                                      SIMDs of a CU hold even shares of the chunks (the
                                      default where that shortens the check phase, for
                                      batches of at least two frames per CU; smaller
                                      batches run variant 0).
                                      Large codes whose checks all have degree 6 or 8
                                      (the LDS accumulator exchange), chunks a wave holds
                                      in registers: streamed form 0 none (every phase
                                      walks the chunks), 1 none (walk one chunk ahead,
                                      the default for degree 8), 2 two; persistent-global
                                      FP32 0 none, 1 none (one ahead), 2 one (default), 3
                                      all, with two of the plan's waves per hardware wave
                                      (degree 6, at most 8 chunks per wave);
                                      persistent-global FP16 0 all (default; at most 8
                                      chunks per wave), 1 four.  -1 otherwise            */
} lpdec_launch_info;

/* The launch a decode of `code` with parameters `p` (NULL = defaults; mode and
 * storage matter) would use.  Errors as lpdec_decode's mode resolution. */
lpdec_status lpdec_code_launch_info(const lpdec_code *code, const lpdec_params *p,
                                    lpdec_launch_info *out);

/* Variants a form can have (lpdec_launch_info.variant lies in 0..LPDEC_TUNE_VARIANTS-1). */
#define LPDEC_TUNE_VARIANTS 4

/* Fix the launch of one form (LPDEC_MODE_RESIDENT, _STREAMED or
 * _PERSISTENT_GLOBAL) for this code.
 *   blocks_per_cu  workgroups per CU, 1..32; 0 restores the runtime's estimate
 *   variant        see lpdec_launch_info.variant, -1..LPDEC_TUNE_VARIANTS-1.
 *                  Streamed form: 0, 1 or 2; a variant the code does not allow
 *                  falls back to the next lower one; -1 restores the default (the
 *                  highest allowed).  Resident form: 0 one frame per workgroup; 1
 *                  two frames per workgroup for every batch size (0 where the code
 *                  does not allow it); -1 restores the default (two frames where
 *                  they help, for batches of at least two frames per CU).  Large
 *                  codes with the accumulator exchange: the held-chunk candidate
 *                  (clamped to the last one the code allows).  Ignored by the
 *                  persistent-global form of other codes.
 * Not synchronised with decodes running on other threads. */
lpdec_status lpdec_code_set_tuning(lpdec_code *code, int32_t mode, int32_t blocks_per_cu,
                                   int32_t variant);

/* Streamed form: issue each block of 16 iteration launches as one replay of a
 * captured HIP graph (enable = 1) instead of 16 kernel launches (enable = 0, the
 * default).  The graph holds kernel nodes only -- the decode launch and a
 * one-thread kernel that advances the launch index the decode reads from device
 * memory -- and is captured and instantiated on first use for a set of launch
 * arguments, then cached with the code's workspace and replayed while the
 * arguments (buffers, batch, parameters, launch shape) stay the same.  A replay may
 * run launches past max_iter, which find every frame finished and do nothing.
 * Results are the same either way.  Not synchronised with decodes on other
 * threads. */
lpdec_status lpdec_code_set_graph(lpdec_code *code, int32_t enable);

/* Autotuner: decode the caller's sample batch (device llr [batch*n]) with
 * parameters `p` once per candidate launch -- workgroups per CU 1..max_blocks_per_cu,
 * times the variants the code allows (streamed form: 0, 1, 2; resident form: 0, 1
 * where two frames per workgroup are possible) -- after one
 * untimed warm-up decode, time each with HIP events on `stream`, and keep the
 * fastest for the form `p` resolves to.  Synchronous.
 *   best_out  host [2], may be NULL: the chosen blocks_per_cu and variant (-1
 *             for forms without variants)
 *   ms_out    host [LPDEC_TUNE_VARIANTS*max_blocks_per_cu], may be NULL: time of candidate
 *             (variant v, blocks b) at [v*max_blocks_per_cu + b - 1] (forms with
 *             variants), or at [b - 1] (others); -1 where not run
 * Scratch outputs are allocated and freed inside the call. */
lpdec_status lpdec_autotune(lpdec_code *code, int32_t batch, const float *llr, const lpdec_params *p,
                            int32_t max_blocks_per_cu, int32_t *best_out, float *ms_out, void *stream);

/* Autotuner for lpdec_decode_multi: decode the caller's sample set (laid out as for
 * lpdec_decode_multi, x written at the LLR offsets into a scratch buffer) once per
 * candidate of the fused persistent launch -- the form (RESIDENT when every code
 * fits it, PERSISTENT_GLOBAL) x workgroups per CU 1..max_blocks_per_cu x the order
 * frames are handed out (1: frames of larger codes first, 0: submission order) --
 * after one untimed warm-up per form and order, timing each with HIP events on
 * `stream`; the fastest becomes the tuning of the set's leading code codes[0]
 * (workgroups per CU of that form and the frame order; multi-code launches take
 * their tuning from codes[0]).  p must ask for mode AUTO and FP32 storage; later
 * decodes pass mode = best_out[0].  Results do not depend on any of these choices.
 *   best_out  host [3], may be NULL: {mode, blocks_per_cu, order}
 *   ms_out    host [4*max_blocks_per_cu], may be NULL: time of (form f, order o,
 *             blocks b) at [(2 f + o) * max_blocks_per_cu + b - 1], f = 0 resident,
 *             1 persistent-global; -1 where not run
 * Synchronous; scratch outputs are allocated and freed inside the call. */
lpdec_status lpdec_autotune_multi(const lpdec_code *const *codes, int32_t ncodes, int32_t nframes,
                                  const int32_t *code_of_frame, const int64_t *llr_offset,
                                  const float *llr, int64_t llr_len, const lpdec_params *p,
                                  int32_t max_blocks_per_cu, int32_t *best_out, float *ms_out,
                                  void *stream);

/* The check-node operation alone: z_k = Pi_PPd(v_k) for `count` vectors of
 * degree d (2 <= d <= LPDEC_MAX_CHECK_DEGREE), Algorithm 2 / Sec. 4.4.
 *   v, z  device [count*d] FP32, row-major (z may not alias v).  Entries of v
 *         must be finite; the result for a vector holding a NaN or an infinity
 *         is unspecified. */
lpdec_status lpdec_project(int32_t d, int32_t count, const float *v, float *z, void *stream);

/* ------------------------------------------------------------------------- */
/* Serving: a request loop with continuous batching.
 *
 * Requests (frames of one code) are submitted from host memory at any time.  A
 * dispatcher thread admits them in arrival order while their device footprint
 * fits the budget, stages their LLRs into HBM and launches them on one of
 * `max_inflight` streams, so requests that arrive while others are decoding start
 * as soon as a stream and memory are free and run concurrently with them.
 * budget_bytes bounds all device memory the server allocates: each launch slot
 * owns a scratch region (queue counter, per-frame metadata and the persistent
 * forms' per-workgroup state), sized at creation for a launch of max_batch_frames
 * frames of the most demanding code at its full grid but to at most half the
 * budget over all slots (a slot then runs fewer workgroups at once; results do
 * not change), and the rest is the LLR arena, of which each admitted frame holds
 * 4 n bytes until its request completes.  The dispatcher allocates nothing.  Each frame's completion is signalled by the kernel
 * itself, so a request completes when its own frames do, not when its launch
 * does.  Codes stay resident; a frame's result is the same alone or in the mix.
 * Latency = submit to host-visible result. */
typedef struct lpdec_server lpdec_server;

#define LPDEC_EXECUTOR_GPU 0
#define LPDEC_EXECUTOR_HOST_NULL 1 /* host-only executor for testing the scheduler without
                                      a GPU: frames complete at once with x = 1/2,
                                      iters = 0, flags = 0 (nothing is decoded)         */

typedef struct {
    int64_t budget_bytes;     /* device bytes for admitted frames (> 0)                 */
    int32_t max_batch_frames; /* frames per launch (>= 1)                               */
    int32_t max_inflight;     /* launches in flight at once (1..8; default 8)           */
    int32_t max_pending;      /* queued requests before submit returns LPDEC_EBUSY      */
    int32_t executor;         /* LPDEC_EXECUTOR_*                                       */
} lpdec_server_config;

lpdec_server_config lpdec_server_default_config(void);

/* codes: host [ncodes] code handles (GPU executor), or NULL with code_n: host [ncodes]
 * code lengths (host-null executor only).  p: NULL = lpdec_default_params(); only the
 * resident and persistent-global forms (FP32) serve.  The server keeps pointers to the
 * codes: destroy the server before its codes.  Errors: LPDEC_EINVAL (also a budget
 * too small for the launch slots' scratch and one frame of the shortest code),
 * LPDEC_ENOMEM, LPDEC_EDEVICE, LPDEC_EUNSUPPORTED. */
lpdec_status lpdec_server_create(const lpdec_code *const *codes, const int32_t *code_n, int32_t ncodes,
                                 const lpdec_params *p, const lpdec_server_config *cfg,
                                 lpdec_server **out);

/* Submit `frames` frames of code `code`; llr is host [frames*n] FP32, copied before
 * return.  *ticket identifies the request.  Errors: LPDEC_EINVAL (bad code or frame
 * count, or a request larger than the whole LLR arena), LPDEC_EBUSY (max_pending
 * queued). */
lpdec_status lpdec_server_submit(lpdec_server *s, int32_t code, int32_t frames, const float *llr,
                                 int64_t *ticket);

#define LPDEC_REQ_QUEUED 0
#define LPDEC_REQ_RUNNING 1
#define LPDEC_REQ_DONE 2
lpdec_status lpdec_server_poll(lpdec_server *s, int64_t ticket, int32_t *state);

/* Wait up to timeout_s (< 0: forever) for a request, copy its results into host
 * buffers (x [frames*n], iters [frames], flags [frames]; any may be NULL) and release
 * it.  latency_s (may be NULL) receives submit-to-completion time.  LPDEC_EBUSY on
 * timeout (the request stays live); LPDEC_EINVAL for an unknown ticket. */
lpdec_status lpdec_server_wait(lpdec_server *s, int64_t ticket, double timeout_s, float *x, int32_t *iters,
                               uint8_t *flags, double *latency_s);

/* Withdraw a request that is still queued; LPDEC_EBUSY once it has been admitted. */
lpdec_status lpdec_server_cancel(lpdec_server *s, int64_t ticket);

typedef struct {
    int64_t submitted, completed, cancelled, rejected;
    int64_t frames_completed, bits_completed; /* coded bits */
    int64_t inflight_bytes, peak_bytes;        /* LLR arena held by admitted frames: now, maximum */
    int64_t launches;
    int32_t queued, running;
    double p50_latency_s, p99_latency_s, mean_latency_s, max_latency_s;
    double elapsed_s;                          /* first submit to last completion */
    int64_t workspace_bytes;                   /* launch slots' scratch (fixed at creation)      */
    int64_t peak_device_bytes;                 /* workspace_bytes + peak_bytes (<= budget_bytes) */
    int32_t peak_concurrent_launches;          /* launches in flight at once, at most            */
} lpdec_server_stats;

lpdec_status lpdec_server_get_stats(lpdec_server *s, lpdec_server_stats *st);

/* Stop the dispatcher: running launches finish, queued requests are dropped.  NULL-safe. */
void lpdec_server_destroy(lpdec_server *s);

/* Message for the last failed call on this thread ("" if none). */
const char *lpdec_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LPDEC_H */
