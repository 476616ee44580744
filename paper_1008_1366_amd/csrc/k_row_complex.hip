// Instantiations of the complex implicit and plain cyclic row kernels.
#include "launch.hpp"
#include "runtime.hpp"

namespace impconv {

template <typename T, int N>
static hipError_t go_complex(const RowArgs& a, hipStream_t s)
{
    constexpr int threads = row_block<T>(N);
    const int64_t blocks = (a.nrows + row_GPB<T>(N) - 1) / row_GPB<T>(N);
    if (blocks == 0) return hipSuccess;
    if constexpr (complex_serial<T, N>()) {
        if (a.M == 1) {
            // one row per 1024-thread workgroup, residues one after the other
            timing_begin(s);
            hipLaunchKernelGGL((k_conv1d_complex_serial<T, N>), dim3(a.nrows), dim3(1024), 0, s, a);
            timing_end("k_conv1d_complex", s);
            return hipGetLastError();
        }
    }
    if (a.M == 1) {
        constexpr bool accg = !regs_fit<T>(3, fft_E<T>(N), threads);
        timing_begin(s);
        hipLaunchKernelGGL((k_conv1d_complex<T, N, accg, false>), dim3(blocks), dim3(threads), 0, s, a);
        timing_end("k_conv1d_complex", s);
    } else {
        constexpr bool accg = !regs_fit<T>(4, fft_E<T>(N), threads);
        timing_begin(s);
        hipLaunchKernelGGL((k_conv1d_complex<T, N, accg, true>), dim3(blocks), dim3(threads), 0, s, a);
        timing_end("k_conv1d_complex", s);
    }
    return hipGetLastError();
}

template <typename T, int N>
static hipError_t go_cyclic(const RowArgs& a, hipStream_t s)
{
    const int64_t blocks = (a.nrows + row_GPB<T>(N) - 1) / row_GPB<T>(N);
    if (blocks == 0) return hipSuccess;
    timing_begin(s);
        hipLaunchKernelGGL((k_conv1d_cyclic<T, N>), dim3(blocks), dim3(row_block<T>(N)), 0, s, a);
        timing_end("k_conv1d_cyclic", s);
    return hipGetLastError();
}

hipError_t launch_row_complex(int dt, int N, const RowArgs& a, hipStream_t s)
{
    if (dt == 0 && (a.flags & kComp)) return launch_row_complex_comp(N, a, s);
    switch (N) {
#define X(n) case n: return dt ? go_complex<double, n>(a, s) : go_complex<float, n>(a, s);
        IMPCONV_POW2_CASES(X)
#undef X
    }
    return hipErrorInvalidValue;
}

hipError_t launch_row_cyclic(int dt, int N, const RowArgs& a, hipStream_t s)
{
    switch (N) {
#define X(n) case n: return dt ? go_cyclic<double, n>(a, s) : go_cyclic<float, n>(a, s);
        IMPCONV_POW2_CASES(X)
#undef X
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
