// Instantiations of the elementwise pad / crop kernel and the column-pass
// dispatcher.
#include "colpass.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace impconv {

hipError_t launch_pad_rows(int dt, const void* src, void* dst, int64_t nrows, int64_t src_ld,
                           int64_t copy, int64_t dst_ld, hipStream_t s)
{
    const int64_t total = nrows * dst_ld;
    if (total == 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    timing_begin(s);
    if (dt)
        hipLaunchKernelGGL(k_pad_rows<double>, dim3(blocks), dim3(256), 0, s, (const C<double>*)src,
                           (C<double>*)dst, nrows, src_ld, copy, dst_ld);
    else
        hipLaunchKernelGGL(k_pad_rows<float>, dim3(blocks), dim3(256), 0, s, (const C<float>*)src,
                           (C<float>*)dst, nrows, src_ld, copy, dst_ld);
    timing_end("k_pad_rows", s);
    return hipGetLastError();
}

hipError_t launch_copy2d(int dt, const void* src, void* dst, int64_t nb, int64_t nsub, int64_t sbs,
                         int64_t sbs2, int64_t sld, int64_t dbs, int64_t dbs2, int64_t dld, int64_t cx,
                         int64_t cy, int64_t dx, int64_t dy, hipStream_t s)
{
    const int64_t total = nb * dx * dy;
    if (total == 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 1 << 20) blocks = 1 << 20;
    timing_begin(s);
    if (dt)
        hipLaunchKernelGGL(k_copy2d<double>, dim3(blocks), dim3(256), 0, s, (const C<double>*)src,
                           (C<double>*)dst, nb, nsub, sbs, sbs2, sld, dbs, dbs2, dld, cx, cy, dx, dy);
    else
        hipLaunchKernelGGL(k_copy2d<float>, dim3(blocks), dim3(256), 0, s, (const C<float>*)src,
                           (C<float>*)dst, nb, nsub, sbs, sbs2, sld, dbs, dbs2, dld, cx, cy, dx, dy);
    timing_end("k_copy2d", s);
    return hipGetLastError();
}

hipError_t launch_col(int dt, int N, int mode, int dir, const ColArgs& a, hipStream_t s)
{
    switch (mode) {
        case kPadBwd:
        case kPadFwd: return launch_col_pad(dt, N, mode, a, s);
        case kCenBwd:
        case kCenFwd: return launch_col_cen(dt, N, mode, a, s);
        case kTerBwd:
        case kTerFwd: return launch_col_ter(dt, N, mode, a, s);
        case kFft: return launch_col_fft(dt, N, dir, a, s);
        case kFsBwd:
        case kFsFwd: return launch_col_fs(dt, N, mode, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
