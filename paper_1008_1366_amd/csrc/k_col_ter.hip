// Instantiations of the kTerBwd / kTerFwd column passes (centered ternary rule, Sec. 4.1).
#include "colpass.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace impconv {

template <typename T, int N, int MODE>
static hipError_t go(const ColArgs& a, hipStream_t s)
{
    const int64_t nb = a.nslab * ((a.ncols + col_TC<T>(N) - 1) / col_TC<T>(N));
    if (nb == 0) return hipSuccess;
    timing_begin(s);
    hipLaunchKernelGGL((k_colpass<T, N, MODE, 1>), dim3(((nb + 7) / 8) * 8), dim3(col_block<T>(N)), 0, s, a);
    timing_end(MODE_NAME(MODE), s);
    return hipGetLastError();
}

hipError_t launch_col_ter(int dt, int N, int mode, const ColArgs& a, hipStream_t s)
{
    switch (N) {
#define X(n) case n: return mode == kTerBwd ? (dt ? go<double, n, kTerBwd>(a, s) : go<float, n, kTerBwd>(a, s)) \
                                        : (dt ? go<double, n, kTerFwd>(a, s) : go<float, n, kTerFwd>(a, s));
        IMPCONV_COL_CASES(X)
#undef X
        // complex64 tconv2 with m_x up to 4096: tiles of two columns
        case 8192: return dt ? hipErrorInvalidValue : (mode == kTerBwd ? go<float, 8192, kTerBwd>(a, s)
                                                                     : go<float, 8192, kTerFwd>(a, s));
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
