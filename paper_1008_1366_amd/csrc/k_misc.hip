// Instantiations of the elementwise pad / crop kernel and the column-pass
// dispatcher.
#include "colpass.hpp"
#include "launch.hpp"

namespace impconv {

hipError_t launch_pad_rows(int dt, const void* src, void* dst, int64_t nrows, int64_t src_ld,
                           int64_t copy, int64_t dst_ld, hipStream_t s)
{
    const int64_t total = nrows * dst_ld;
    if (total == 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (dt)
        hipLaunchKernelGGL(k_pad_rows<double>, dim3(blocks), dim3(256), 0, s, (const C<double>*)src,
                           (C<double>*)dst, nrows, src_ld, copy, dst_ld);
    else
        hipLaunchKernelGGL(k_pad_rows<float>, dim3(blocks), dim3(256), 0, s, (const C<float>*)src,
                           (C<float>*)dst, nrows, src_ld, copy, dst_ld);
    return hipGetLastError();
}

hipError_t launch_col(int dt, int N, int mode, int dir, const ColArgs& a, hipStream_t s)
{
    switch (mode) {
        case kPadBwd:
        case kPadFwd: return launch_col_pad(dt, N, mode, a, s);
        case kCenBwd:
        case kCenFwd: return launch_col_cen(dt, N, mode, a, s);
        case kFft: return launch_col_fft(dt, N, dir, a, s);
        case kFsBwd:
        case kFsFwd: return launch_col_fs(dt, N, mode, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
