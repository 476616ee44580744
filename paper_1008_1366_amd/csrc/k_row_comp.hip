// Instantiations of the complex64 row kernel with compensated twiddle
// products (each product by a root of unity formed from its FP32 high and
// low parts).
#include "launch.hpp"
#include "runtime.hpp"

namespace impconv {

template <int N>
static hipError_t go_complex_comp(const RowArgs& a, hipStream_t s)
{
    using T = float;
    constexpr int threads = row_block<T>(N);
    const int64_t blocks = (a.nrows + row_GPB<T>(N) - 1) / row_GPB<T>(N);
    if (blocks == 0) return hipSuccess;
    if (a.M == 1) {
        constexpr bool accg = !regs_fit<T>(3, fft_E<T>(N), threads);
        timing_begin(s);
        hipLaunchKernelGGL((k_conv1d_complex<T, N, accg, false, true>), dim3(blocks), dim3(threads), 0, s, a);
        timing_end("k_conv1d_complex", s);
    } else {
        constexpr bool accg = !regs_fit<T>(4, fft_E<T>(N), threads);
        timing_begin(s);
        hipLaunchKernelGGL((k_conv1d_complex<T, N, accg, true, true>), dim3(blocks), dim3(threads), 0, s, a);
        timing_end("k_conv1d_complex", s);
    }
    return hipGetLastError();
}

hipError_t launch_row_complex_comp(int N, const RowArgs& a, hipStream_t s)
{
    if (!a.twlo) return hipErrorInvalidValue;
    switch (N) {
#define X(n) case n: return go_complex_comp<n>(a, s);
        IMPCONV_POW2_CASES(X)
#undef X
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
