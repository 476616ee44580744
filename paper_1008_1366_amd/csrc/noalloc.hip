// noalloc.hip -- the allocation-free form of impconv_conv2d.
//
// Callers that cannot allocate device memory (code under hipGraph capture,
// tight serving loops, harnesses that forbid hipMalloc) still need the work
// arrays that the 2D convolution keeps apart from its data (Sec. 1: data and
// work memory are decoupled; Secs. 3.1-3.2: the residue arrays of the outer
// pass).  Here those arrays live in one array of fixed size that is part of
// the library's device code: each device that loads the library holds its
// own copy, allocated with the code object and kept until the process ends.
//
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address).  impconv_init() resolves the device
// address of the current device's copy once, with hipGetSymbolAddress, and
// the entry point hands that address to the kernels as their work pointer.
#include <mutex>
#include <string>

#include "runtime.hpp"

namespace impconv {

// Work memory of impconv_conv2d_noalloc on each device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex s_mu;
void* s_addr[kMaxDevices];  // device address of `scratch`, per device (nullptr: not resolved)
}  // namespace

// Resolves the device address of `scratch` on the current device (once per
// device; thread-safe).  Called by impconv_init().
impconv_status noalloc_setup()
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return hip_fail(hipErrorInvalidDevice, "work memory of the allocation-free entry point");
    std::lock_guard<std::mutex> lk(s_mu);
    if (s_addr[dev]) return IMPCONV_OK;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (work memory of the allocation-free entry point)");
    if (!p) return fail(IMPCONV_E_HIP, "hipGetSymbolAddress returned a null address");
    s_addr[dev] = p;
    return IMPCONV_OK;
}

}  // namespace impconv

using namespace impconv;

extern "C" {

size_t impconv_noalloc_capacity(void) { return kScratchBytes; }

impconv_status impconv_conv2d_noalloc(int kind, int dtype, int64_t batch, int64_t M, const int64_t* m,
                                      const int64_t* n, const void* f, const void* g, void* h,
                                      uint32_t flags, void* stream)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    void* w = nullptr;
    if (dev >= 0 && dev < kMaxDevices) {
        std::lock_guard<std::mutex> lk(s_mu);
        w = s_addr[dev];
    }
    if (!w) return fail(IMPCONV_E_ARG, "impconv_init() has not run on this device (it resolves the work memory "
                                       "of the allocation-free entry point)");
    size_t need = 0;
    impconv_status st = impconv_convnd_workspace(kind, dtype, 2, m, n, batch, M, flags, &need);
    if (st) return st;
    if (need > kScratchBytes)
        return fail(IMPCONV_E_WORKSPACE, "this convolution needs " + std::to_string(need) +
                                             " bytes of work memory; the allocation-free entry point has " +
                                             std::to_string(kScratchBytes));
    // every kernel of the 2D path writes each element of its work arrays
    // before reading it, so nothing left by an earlier call needs clearing
    return impconv_conv2d(kind, dtype, batch, M, m, n, f, g, h, w, kScratchBytes, flags, stream);
}

}  // extern "C"
