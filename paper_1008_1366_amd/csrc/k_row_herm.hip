// Instantiations of the centered Hermitian (2/3 rule) and ternary row kernels.
#include "launch.hpp"
#include "runtime.hpp"

namespace impconv {

template <typename T, int NC>
static hipError_t go_herm(const RowArgs& a, hipStream_t s)
{
    constexpr int threads = row_block<T, 1>(NC);
    const int64_t blocks = (a.nrows + row_GPB<T, 1>(NC) - 1) / row_GPB<T, 1>(NC);
    if (blocks == 0) return hipSuccess;
    timing_begin(s);
    // in place (the staged kernel accumulates its output in h): the
    // register-resident kernel, which reads every input before it stores
    const bool inplace = a.h == a.f || a.h == a.g;
    if constexpr (herm_staged<T, NC>()) {
        if (inplace) {
            if (a.M == 1)
                hipLaunchKernelGGL((k_conv1d_hermitian<T, NC, false>), dim3(blocks), dim3(threads), 0, s, a);
            else
                hipLaunchKernelGGL((k_conv1d_hermitian<T, NC, true>), dim3(blocks), dim3(threads), 0, s, a);
            timing_end("k_conv1d_hermitian", s);
            return hipGetLastError();
        }
    }
    if constexpr (herm_staged<T, NC>()) {
        // one row per 1024-thread workgroup, residues one at a time
        const dim3 st(kHermStagedThreads);
        if (a.M == 1)
            hipLaunchKernelGGL((k_conv1d_hermitian_staged<T, NC, false>), dim3(a.nrows), st, 0, s, a);
        else
            hipLaunchKernelGGL((k_conv1d_hermitian_staged<T, NC, true>), dim3(a.nrows), st, 0, s, a);
    } else {
        if (a.M == 1)
            hipLaunchKernelGGL((k_conv1d_hermitian<T, NC, false>), dim3(blocks), dim3(threads), 0, s, a);
        else
            hipLaunchKernelGGL((k_conv1d_hermitian<T, NC, true>), dim3(blocks), dim3(threads), 0, s, a);
    }
    timing_end("k_conv1d_hermitian", s);
    return hipGetLastError();
}

template <typename T, int NN>
static hipError_t go_tern(const RowArgs& a, hipStream_t s)
{
    constexpr int threads = row_block<T, 1>(NN);
    constexpr bool accg = !regs_fit<T>(5, row_E<T, 1>(NN), threads);
    const int64_t blocks = (a.nrows + row_GPB<T, 1>(NN) - 1) / row_GPB<T, 1>(NN);
    if (blocks == 0) return hipSuccess;
    timing_begin(s);
        hipLaunchKernelGGL((k_conv1d_ternary<T, NN, accg>), dim3(blocks), dim3(threads), 0, s, a);
        timing_end("k_conv1d_ternary", s);
    return hipGetLastError();
}

hipError_t launch_row_hermitian(int dt, int NC, const RowArgs& a, hipStream_t s)
{
    switch (NC) {
#define X(n) case n: return dt ? go_herm<double, n>(a, s) : go_herm<float, n>(a, s);
        IMPCONV_POW2_CASES(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename T, int NC>
static hipError_t go_realcyclic(const RowArgs& a, hipStream_t s)
{
    const int64_t blocks = (a.nrows + row_GPB<T, 1>(NC) - 1) / row_GPB<T, 1>(NC);
    if (blocks == 0) return hipSuccess;
    timing_begin(s);
        hipLaunchKernelGGL((k_conv1d_realcyclic<T, NC>), dim3(blocks), dim3(row_block<T, 1>(NC)), 0, s, a);
        timing_end("k_conv1d_realcyclic", s);
    return hipGetLastError();
}

hipError_t launch_row_realcyclic(int dt, int NC, const RowArgs& a, hipStream_t s)
{
    switch (NC) {
#define X(n) case n: return dt ? go_realcyclic<double, n>(a, s) : go_realcyclic<float, n>(a, s);
        IMPCONV_POW2_CASES(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename T, int NN>
static bool tern_accumulates()
{
    return !regs_fit<T>(5, row_E<T, 1>(NN), row_block<T, 1>(NN));
}

bool row_ternary_accumulates(int dt, int NN)
{
    switch (NN) {
#define X(n) case n: return dt ? tern_accumulates<double, n>() : tern_accumulates<float, n>();
        IMPCONV_POW2_CASES(X)
#undef X
    }
    return true;
}

hipError_t launch_row_ternary(int dt, int NN, const RowArgs& a, hipStream_t s)
{
    switch (NN) {
#define X(n) case n: return dt ? go_tern<double, n>(a, s) : go_tern<float, n>(a, s);
        IMPCONV_POW2_CASES(X)
#undef X
    }
    return hipErrorInvalidValue;
}

}  // namespace impconv
