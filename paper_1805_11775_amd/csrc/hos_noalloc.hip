// hos_noalloc.hip -- hos_bispectrum on a fixed device scratch array, for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The workspace of hos_bispectrum lives here in a file-scope device array of
// HOS_NOALLOC_SCRATCH_BYTES.  Every device the library runs on holds its own
// copy of the array, at its own address, until the process ends.  In host
// code the array's name is only a host-side stand-in, so its device address
// is looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is ever handed to kernels.
//
// The kernels of hos_bispectrum need no part of the workspace to start at
// zero (every value they read was written earlier in the same call), so the
// array is never cleared.  All calls on one device share the array: calls
// that overlap in time on one device (different streams, or different host
// threads without ordering) race on it and must be serialised by the caller.
#include <mutex>

#include "hos_internal.h"

namespace hos {
namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[HOS_NOALLOC_SCRATCH_BYTES];

std::mutex scratch_mu;
void *scratch_ptr[NOALLOC_MAX_DEVICES];

// Device address of the current device's scratch array (looked up on the
// first call on that device), or NULL with *st set.
void *scratch_for_current_device(int *st)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        *st = HOS_ENODEVICE;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            *st = HOS_EDEVICE;
            return nullptr;
        }
        scratch_ptr[dev] = ptr;
    }
    *st = HOS_OK;
    return scratch_ptr[dev];
}

}  // namespace
}  // namespace hos

extern "C" int hos_bispectrum_noalloc(const void *x, int32_t dtype, int64_t n, int32_t M,
                                      int32_t window, int32_t nfft, int32_t path,
                                      uint32_t flags, double *c3, double *B,
                                      hipStream_t stream)
{
    // argument checks and the scratch bound first, on the host: a rejected
    // call makes no HIP call
    hos::C3Plan p;
    int st = hos::bispectrum_check(x, dtype, n, M, window, nfft, path, flags, c3, B, p);
    if (st != HOS_OK)
        return st;
    if (p.total > HOS_NOALLOC_SCRATCH_BYTES)
        return HOS_ESCRATCH;
    st = hos::device_ok_public();
    if (st != HOS_OK)
        return st;
    void *ws = hos::scratch_for_current_device(&st);
    if (!ws)
        return st;
    return hos::bispectrum_run(x, dtype, n, M, window, nfft, path, flags, c3, B, ws,
                               HOS_NOALLOC_SCRATCH_BYTES, stream, nullptr);
}
