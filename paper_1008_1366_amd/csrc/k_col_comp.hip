// Instantiations of the complex64 kPadBwd / kPadFwd column passes with
// compensated twiddle products (one workgroup per tile).
#include "colpass.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace impconv {

template <int N, int MODE>
static hipError_t go_comp(const ColArgs& a, hipStream_t s)
{
    using T = float;
    const int64_t nb = a.nslab * ((a.ncols + col_TC<T>(N) - 1) / col_TC<T>(N));
    if (nb == 0) return hipSuccess;
    timing_begin(s);
    hipLaunchKernelGGL((k_colpass<T, N, MODE, 1, true>), dim3(((nb + 7) / 8) * 8), dim3(col_block<T>(N)), 0, s, a);
    timing_end(MODE_NAME(MODE), s);
    return hipGetLastError();
}

hipError_t launch_col_pad_comp(int N, int mode, const ColArgs& a, hipStream_t s)
{
    if (!a.twlo) return hipErrorInvalidValue;
    switch (N) {
#define X(n) case n: return mode == kPadBwd ? go_comp<n, kPadBwd>(a, s) : go_comp<n, kPadFwd>(a, s);
        IMPCONV_COL_CASES(X)
#undef X
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
