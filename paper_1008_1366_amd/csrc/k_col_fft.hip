// Instantiations of the plain strided FFT column pass (explicit comparator).
#include "colpass.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace impconv {

template <typename T, int N, int DIR>
static hipError_t go(const ColArgs& a, hipStream_t s)
{
    const int64_t nb = a.nslab * ((a.ncols + col_TC<T>(N) - 1) / col_TC<T>(N));
    if (nb == 0) return hipSuccess;
    timing_begin(s);
    hipLaunchKernelGGL((k_colpass<T, N, kFft, DIR>), dim3(((nb + 7) / 8) * 8), dim3(col_block<T>(N)), 0, s, a);
    timing_end(MODE_NAME(kFft), s);
    return hipGetLastError();
}

hipError_t launch_col_fft(int dt, int N, int dir, const ColArgs& a, hipStream_t s)
{
    switch (N) {
#define X(n) case n: return dir > 0 ? (dt ? go<double, n, 1>(a, s) : go<float, n, 1>(a, s)) \
                                    : (dt ? go<double, n, -1>(a, s) : go<float, n, -1>(a, s));
        IMPCONV_COL_CASES(X)
#undef X
        // the explicit tconv2 comparator's x transform at m_x up to 4096
        // (complex64: tiles of two and one columns)
        case 8192: return dt ? hipErrorInvalidValue : (dir > 0 ? go<float, 8192, 1>(a, s) : go<float, 8192, -1>(a, s));
        case 16384: return dt ? hipErrorInvalidValue : (dir > 0 ? go<float, 16384, 1>(a, s) : go<float, 16384, -1>(a, s));
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
