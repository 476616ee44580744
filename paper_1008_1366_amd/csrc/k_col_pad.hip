// Instantiations of the kPadBwd / kPadFwd column passes.
#include "colpass.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace impconv {

// Byte offsets of the pipelined kernel's buffer accesses within one tile
// (columns < TC, rows < N) must stay below the resource's record count.
template <typename T, int N>
static bool pipe_offsets_fit(int64_t ld)
{
    const int64_t hi = (int64_t(col_TC<T>(N)) + int64_t(N - 1) * ld + 1) * int64_t(sizeof(C<T>));
    return hi <= int64_t(kBufRecords);
}

template <typename T, int N, int MODE>
static hipError_t go(const ColArgs& a, hipStream_t s)
{
    const int64_t nb = a.nslab * ((a.ncols + col_TC<T>(N) - 1) / col_TC<T>(N));
    if (nb == 0) return hipSuccess;
    if constexpr (pipe_ok<T>(N)) {
        // one persistent workgroup per CU (the LDS holds one tile), at least
        // two tiles each; one set of slabs only (k_colpipe has no second set)
        const int64_t grid = int64_t(a.ncu) / 8 * 8;
        if (a.nslab2 == 0 && grid >= 8 && nb >= 2 * grid && pipe_offsets_fit<T, N>(a.in_ld) &&
            pipe_offsets_fit<T, N>(a.out_ld)) {
            timing_begin(s);
            hipLaunchKernelGGL((k_colpipe<T, N, MODE>), dim3(grid), dim3(col_block<T>(N)), 0, s, a);
            timing_end(MODE_NAME(MODE), s);
            return hipGetLastError();
        }
    }
    timing_begin(s);
    hipLaunchKernelGGL((k_colpass<T, N, MODE, 1>), dim3(((nb + 7) / 8) * 8), dim3(col_block<T>(N)), 0, s, a);
    timing_end(MODE_NAME(MODE), s);
    return hipGetLastError();
}

hipError_t launch_col_pad(int dt, int N, int mode, const ColArgs& a, hipStream_t s)
{
    if (dt == 0 && (a.fsflags & 8)) return launch_col_pad_comp(N, mode, a, s);
    switch (N) {
#define X(n) case n: return mode == kPadBwd ? (dt ? go<double, n, kPadBwd>(a, s) : go<float, n, kPadBwd>(a, s)) \
                                        : (dt ? go<double, n, kPadFwd>(a, s) : go<float, n, kPadFwd>(a, s));
        IMPCONV_COL_CASES(X)
#undef X
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
