// C ABI of the auxiliary kernels: dual subgradient decoding (Appendix A) and
// the per-frame ML lower-bound bookkeeping (Sec. 5.1).
#include <cmath>
#include <cstring>

#include "lpdec_aux.h"
#include "lpdec_runtime.h"

using namespace lpdec;

#define fail lpdec_fail
#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            return fail(LPDEC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

namespace {

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 256;
    return cus;
}

lpdec_status check_device(const lpdec_code *code) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (code->device != dev)
        return fail(LPDEC_EINVAL, "code was created on device %d, current device is %d", code->device, dev);
    return LPDEC_OK;
}

}  // namespace

extern "C" {

lpdec_status lpdec_decode_dual(const lpdec_code *code, int32_t batch, const float *llr, const lpdec_params *pin,
                               float *x_out, int32_t *iters_out, uint8_t *flags_out, void *stream_v) {
    if (!code) return fail(LPDEC_EINVAL, "code must not be NULL");
    lpdec_params p = pin ? *pin : lpdec_default_params();
    if (!(p.mu > 0.0f) || !std::isfinite(p.mu)) return fail(LPDEC_EINVAL, "mu (the step size) must be positive");
    if (p.max_iter < 1) return fail(LPDEC_EINVAL, "max_iter must be >= 1");
    if (batch < 0) return fail(LPDEC_EINVAL, "batch must be >= 0");
    if (batch == 0) return LPDEC_OK;
    if (!llr || !x_out || !iters_out || !flags_out)
        return fail(LPDEC_EINVAL, "llr, x_out, iters_out and flags_out must not be NULL");
    const DevCode &D = code->dc;
    if (D.cpt > 8) return fail(LPDEC_EUNSUPPORTED, "dual decoding holds at most 8 check chunks per wave");
    if (D.dmax > 8) return fail(LPDEC_EUNSUPPORTED, "dual decoding supports check degrees up to 8 (code has %d)", D.dmax);
    DualLaunch L{};
    L.dclass = (D.dmin == 6 && D.dmax == 6) ? 0 : 1;
    L.cpt = D.cpt;
    L.threads = D.waves * kWave;
    L.lds_bytes = ((size_t)9 * D.n + 15) / 16 * 16;
    if (L.lds_bytes > 160 * 1024) return fail(LPDEC_EUNSUPPORTED, "dual decoding needs 9 n bytes of LDS, n is too large");
    lpdec_status st = check_device(code);
    if (st != LPDEC_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    int per_cu = 0;
    FrameBatch fb{};
    if (launch_dual(L, code->d_dc, fb, 0.0, 0, stream, &per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
    L.grid = std::max(1, std::min<int>(batch, device_cus() * per_cu));
    Workspace &ws = const_cast<lpdec_code *>(code)->ws;
    WsGuard guard(ws, stream);
    HIP_TRY(ws.queue.ensure(sizeof(int)));
    fb.nframes = batch;
    fb.llr = llr;
    fb.x_out = x_out;
    fb.iters_out = iters_out;
    fb.flags_out = flags_out;
    fb.queue = static_cast<int *>(ws.queue.p);
    HIP_TRY(launch_fill_i32(fb.queue, 0, 1, stream));
    hipError_t e = launch_dual(L, code->d_dc, fb, (double)p.mu, p.max_iter, stream, nullptr);
    if (e != hipSuccess) return fail(LPDEC_EDEVICE, "dual launch failed: %s", hipGetErrorString(e));
    return LPDEC_OK;
}

static lpdec_status evaluate_core(const lpdec_code *const *codes, int ncodes, int nframes, const int32_t *cof,
                                  const int64_t *loff, const int64_t *xoff, const float *llr, const float *x,
                                  const uint8_t *sent, int32_t *bit_errors, double *cost_hat, double *cost_sent,
                                  uint8_t *outcome, void *stream_v) {
    if (nframes < 0) return fail(LPDEC_EINVAL, "nframes must be >= 0");
    if (nframes == 0) return LPDEC_OK;
    if (!llr || !x || !bit_errors || !cost_hat || !cost_sent || !outcome)
        return fail(LPDEC_EINVAL, "llr, x and the four outputs must not be NULL");
    int nmax = 0;
    for (int c = 0; c < ncodes; ++c) {
        lpdec_status st = check_device(codes[c]);
        if (st != LPDEC_OK) return st;
        nmax = std::max(nmax, codes[c]->dc.n);
    }
    if (nmax > 160 * 1024) return fail(LPDEC_EUNSUPPORTED, "code too long for the evaluation kernel");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    EvalBatch eb{};
    eb.nframes = nframes;
    eb.llr = llr;
    eb.x = x;
    eb.sent = sent;
    eb.bit_errors = bit_errors;
    eb.cost_hat = cost_hat;
    eb.cost_sent = cost_sent;
    eb.outcome = outcome;
    const DevCode *codes_dev = codes[0]->d_dc;
    Workspace &ws = const_cast<lpdec_code *>(codes[0])->ws;
    WsGuard guard(ws, stream);
    if (cof || loff || xoff) {
        // per-call metadata through the workspace's pinned staging (the previous
        // call's copy out of it must have finished first)
        const size_t tbl = ((sizeof(DevCode) * ncodes + 255) / 256) * 256;
        const size_t bytes = tbl + (size_t)nframes * (2 * sizeof(int64_t) + sizeof(int32_t));
        if (ws.last) HIP_TRY(hipEventSynchronize(ws.last));
        if (ws.host_meta_bytes < bytes) {
            if (ws.host_meta) HIP_TRY(hipHostFree(ws.host_meta));
            ws.host_meta = nullptr;
            ws.host_meta_bytes = 0;
            HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&ws.host_meta), bytes, hipHostMallocDefault));
            ws.host_meta_bytes = bytes;
        }
        HIP_TRY(ws.frame_meta.ensure(bytes));
        char *h = ws.host_meta;
        for (int c = 0; c < ncodes; ++c) std::memcpy(h + sizeof(DevCode) * c, &codes[c]->dc, sizeof(DevCode));
        int64_t *hl = reinterpret_cast<int64_t *>(h + tbl);
        int64_t *hx = hl + nframes;
        int32_t *hc = reinterpret_cast<int32_t *>(hx + nframes);
        for (int f = 0; f < nframes; ++f) {
            const int c = cof ? cof[f] : 0;
            hl[f] = loff ? loff[f] : (int64_t)f * codes[0]->dc.n;
            hx[f] = xoff ? xoff[f] : (int64_t)f * codes[0]->dc.n;
            hc[f] = c;
        }
        HIP_TRY(hipMemcpyAsync(ws.frame_meta.p, h, bytes, hipMemcpyHostToDevice, stream));
        char *d = static_cast<char *>(ws.frame_meta.p);
        codes_dev = reinterpret_cast<const DevCode *>(d);
        eb.llr_off = reinterpret_cast<const int64_t *>(d + tbl);
        eb.x_off = eb.llr_off + nframes;
        eb.code_of_frame = reinterpret_cast<const int32_t *>(eb.x_off + nframes);
    }
    hipError_t e = launch_evaluate(codes_dev, eb, nmax, stream);
    if (e != hipSuccess) return fail(LPDEC_EDEVICE, "evaluation launch failed: %s", hipGetErrorString(e));
    return LPDEC_OK;
}

lpdec_status lpdec_evaluate(const lpdec_code *code, int32_t batch, const float *llr, const float *x,
                            const uint8_t *sent, int32_t *bit_errors, double *cost_hat, double *cost_sent,
                            uint8_t *outcome, void *stream) {
    if (!code) return fail(LPDEC_EINVAL, "code must not be NULL");
    return evaluate_core(&code, 1, batch, nullptr, nullptr, nullptr, llr, x, sent, bit_errors, cost_hat, cost_sent,
                         outcome, stream);
}

lpdec_status lpdec_evaluate_multi(const lpdec_code *const *codes, int32_t ncodes, int32_t nframes,
                                  const int32_t *code_of_frame, const int64_t *llr_offset, const float *llr,
                                  int64_t llr_len, const float *x, const int64_t *x_offset, int64_t x_len,
                                  const uint8_t *sent, int32_t *bit_errors, double *cost_hat, double *cost_sent,
                                  uint8_t *outcome, void *stream) {
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
            return fail(LPDEC_EINVAL, "frame %d: llr range outside llr_len", f);
        if (x_offset[f] < 0 || x_offset[f] + n > x_len)
            return fail(LPDEC_EINVAL, "frame %d: x range outside x_len", f);
    }
    return evaluate_core(codes, ncodes, nframes, code_of_frame, llr_offset, x_offset, llr, x, sent, bit_errors,
                         cost_hat, cost_sent, outcome, stream);
}

}  // extern "C"
