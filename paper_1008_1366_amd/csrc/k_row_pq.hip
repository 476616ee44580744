// Instantiations of the general p/q padding row kernel (Sec. 2.4).
#include "launch.hpp"
#include "runtime.hpp"

namespace impconv {

template <typename T, int NP, int P>
static hipError_t go_pq(const RowArgs& a, hipStream_t s)
{
    const int64_t blocks = (a.nrows + row_GPB<T, 1>(NP) - 1) / row_GPB<T, 1>(NP);
    if (blocks == 0) return hipSuccess;
    timing_begin(s);
    hipLaunchKernelGGL((k_conv1d_pq<T, NP, P>), dim3(blocks), dim3(row_block<T, 1>(NP)), 0, s, a);
    timing_end("k_conv1d_pq", s);
    return hipGetLastError();
}

template <typename T, int NP>
static hipError_t go_pq_p(int P, const RowArgs& a, hipStream_t s)
{
    switch (P) {
        case 2: return go_pq<T, NP, 2>(a, s);
        case 3: return go_pq<T, NP, 3>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_row_pq(int dt, int NP, int P, const RowArgs& a, hipStream_t s)
{
    switch (NP) {
#define X(n) case n: return dt ? go_pq_p<double, n>(P, a, s) : go_pq_p<float, n>(P, a, s);
        IMPCONV_COL_CASES(X)
#undef X
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
