// Allocation-free decode entry point (lpdec_decode_noalloc, lpdec.h).
//
// Callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid it) still need the decoder's
// scratch: the persistent launch's queue counter and, for some codes, the
// per-workgroup buffers of the persistent forms.  Here that scratch is one
// file-scope device array per GPU, loaded with the library's code object and
// held until the process ends.  Its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is ever
// handed to kernels: in host code the array's name is a host-side stand-in, not
// device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lpdec.h"
#include "lpdec_runtime.h"

namespace {

static __device__ __align__(256) unsigned char scratch[LPDEC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device (nullptr: not looked up yet)

}  // namespace

extern "C" lpdec_status lpdec_decode_noalloc(const lpdec_code *code, int32_t batch, const float *llr,
                                             const lpdec_params *p, float *x_out, int32_t *iters_out,
                                             uint8_t *flags_out, void *stream) {
    if (!code) return lpdec_fail(LPDEC_EINVAL, "code must not be NULL");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return lpdec_fail(LPDEC_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return lpdec_fail(LPDEC_EUNSUPPORTED, "device index %d out of range", dev);
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_scratch[dev]) {
            void *q = nullptr;
            e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !q)
                return lpdec_fail(LPDEC_EDEVICE, "looking up the scratch array on device %d failed: %s", dev,
                                  hipGetErrorString(e));
            g_scratch[dev] = q;
        }
        ptr = g_scratch[dev];
    }
    const ScratchArena arena{static_cast<char *>(ptr), (size_t)LPDEC_NOALLOC_SCRATCH_BYTES};
    return lpdec_decode_core(&code, 1, batch, nullptr, nullptr, nullptr, llr, p, x_out, iters_out, flags_out,
                             nullptr, nullptr, 0, stream, nullptr, nullptr, &arena);
}
