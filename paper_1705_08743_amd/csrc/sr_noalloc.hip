// closure_noalloc: closure() for callers that cannot allocate (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation).  The
// working memory that closure() would allocate stream-ordered -- the binary16
// copy of uint8 data and the two matrices of the squaring closure -- comes
// from `scratch`, a file-scope device array that every device the library
// runs on holds from module load until the process ends.
//
// Host code never passes `scratch` itself (in host code its name stands for a
// host-side shadow, not a device address): on the first call on each device,
// with that device current, hipGetSymbolAddress yields the device copy's
// address, which is kept per device and is what the kernels receive.
//
// Every call on one device shares that device's array and leaves its last
// contents there; the closure clears what must start at zero (the squaring's
// change flags) with a fill kernel on the caller's stream.  Calls whose work
// overlaps in time on one device (several streams, or several host threads)
// race on the array and must be serialized by the caller.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "semiring.h"
#include "sr_internal.h"

static constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_dev_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up once per device.
int scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return sr::report(SR_EDEVICE, "closure_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return sr::report(SR_EUNSUPPORTED, "closure_noalloc: device %d beyond the first %d", dev,
                          kMaxDevices);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_dev_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return sr::report(SR_EDEVICE,
                              "closure_noalloc: hipGetSymbolAddress of the static scratch on "
                              "device %d: %s",
                              dev, hipGetErrorString(e));
        g_dev_ptr[dev] = p;
    }
    *out = g_dev_ptr[dev];
    return SR_OK;
}

}  // namespace

extern "C" {

int closure_noalloc(int kind, void *T, int64_t ldt, int64_t D, unsigned flags, void *stream) {
    return sr::closure_run(kind, T, ldt, D, flags, stream, scratch_ptr, kScratchBytes,
                           "closure_noalloc");
}

}  // extern "C"
