// Instantiations of the kCenBwd / kCenFwd column passes.
#include "colpass.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace impconv {

template <typename T, int N, int MODE>
static hipError_t go(const ColArgs& a, hipStream_t s)
{
    const int64_t nb = a.nslab * ((a.ncols + col_TC<T, MODE>(N) - 1) / col_TC<T, MODE>(N));
    if (nb == 0) return hipSuccess;
    timing_begin(s);
    hipLaunchKernelGGL((k_colpass<T, N, MODE, 1>), dim3(((nb + 7) / 8) * 8), dim3(col_block<T, MODE>(N)), 0, s, a);
    timing_end(MODE_NAME(MODE), s);
    return hipGetLastError();
}

hipError_t launch_col_cen(int dt, int N, int mode, const ColArgs& a, hipStream_t s)
{
    switch (N) {
#define X(n) case n: return mode == kCenBwd ? (dt ? go<double, n, kCenBwd>(a, s) : go<float, n, kCenBwd>(a, s)) \
                                        : (dt ? go<double, n, kCenFwd>(a, s) : go<float, n, kCenFwd>(a, s));
        IMPCONV_COL_CASES(X)
#undef X
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
