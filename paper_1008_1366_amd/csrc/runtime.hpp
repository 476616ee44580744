// runtime.hpp -- host-side internals shared by the C ABI and the kernel
// launch units: per-device twiddle tables, error reporting, launch helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <mutex>
#include <string>

#include "../../include/impconv.h"

namespace impconv {

// Largest power-of-two FFT table (zeta_N^j, N <= 2^kTwLog) and largest N of
// the zeta_{3N}^j tables.
constexpr int kTwLog = 18;
constexpr int kTw3Log = 16;
// General p/q padding (Sec. 2.4): transform sizes NP = 2^l <= 2^kTwqLog,
// residue counts q with a table zeta_{q NP}^j (j < q NP) of their own (the
// power-of-two q use the zeta_N tables).
constexpr int kTwqLog = 12;
constexpr int kTwqList[4] = {3, 5, 6, 7};
// Element offset of zeta_{q NP}^j in the concatenated q tables, or -1.
int64_t twq_off(int q, int64_t NP);

struct DevTables {
    const void* tw[2];   // [0] complex64, [1] complex128: concatenated zeta_N^j, offset N - 1
    const void* tw3[2];  // concatenated zeta_{3N}^j (j < N), offset N - 1
    const void* twq[2];  // concatenated zeta_{q NP}^j (j < q NP), offset twq_off(q, NP)
    const void* twlo;    // complex64 low parts of tw: the FP64 value minus its FP32 rounding, rounded
    const void* tw3lo;   // complex64 low parts of tw3
    int ncu;             // compute units
};

// Tables of the current device, created on first use (FP64 on the host,
// rounded to FP32 for the complex64 copy).  Returns nullptr on HIP failure.
const DevTables* tables();

// Column twiddles of the four-step passes, zeta_F^{j2 c} at [j2][c]
// (j2 < N2, c < N1, F = N1 N2), created on first use per device, dtype and
// split (synchronous; nullptr on HIP failure).
const void* fs_twiddles(int dt, int64_t N2, int64_t N1);

// Auxiliary streams of a device and the events that fork work onto them and
// join it back into the caller's stream: created once, with the first call
// that needs them on the device, and kept until the process ends (no call
// creates or destroys streams).  `mu` is held while a call enqueues through
// them (the events are re-recorded by every call).  Used by ragged batches
// (size classes on separate streams) and by the 3D convolutions (rows of
// one chunk of planes beside the outer pass of the next).
constexpr int kAuxStreams = 3;
struct DevLanes {
    hipStream_t aux[kAuxStreams];
    hipEvent_t fork;
    hipEvent_t join[kAuxStreams];
    hipEvent_t pipe[4];  // 3D pipeline: y stage of a buffer done (0, 1), buffer free again (2, 3)
    std::mutex mu;
};
// The current device's lanes (nullptr with the error set on HIP failure).
DevLanes* device_lanes(int dev);

// Resolves, once per device, the device address of the fixed work memory of
// impconv_conv2d_noalloc on the current device (impconv_init calls it).
impconv_status noalloc_setup();

// FP64 host generation, exposed for the host-side unit test.
void gen_roots(int64_t denom, int64_t count, double* out_re_im);

impconv_status fail(impconv_status st, const std::string& msg);
impconv_status hip_fail(hipError_t e, const char* what);

// Optional per-launch timing (profiling mode, off by default): when enabled,
// every kernel launch of the library is bracketed by two hipEvents recorded
// on its stream; impconv_timing_report aggregates them per kernel name.
bool timing_on();
void timing_begin(hipStream_t s);
void timing_end(const char* name, hipStream_t s);

// Whether output h (nh bytes) overlaps input x (nx bytes) in a way the
// kernels do not support.  h may be x itself when both have the same extent
// (the in-place form): every pass reads its input rows or columns before the
// pass that writes the same elements, and no launch writes data another
// workgroup of it still reads.
inline bool bad_alias(const void* h, size_t nh, const void* x, size_t nx)
{
    if (!h || !x || nh == 0 || nx == 0) return false;
    if (h == x && nh == nx) return false;
    const char* a = static_cast<const char*>(h);
    const char* b = static_cast<const char*>(x);
    return a < b + nx && b < a + nh;
}

inline int64_t next_pow2(int64_t x)
{
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}
inline int ilog2(int64_t x)
{
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

}  // namespace impconv
