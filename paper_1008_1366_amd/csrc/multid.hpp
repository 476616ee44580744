// multid.hpp -- host orchestration of the multi-pass convolutions: 1D
// complex convolutions longer than one workgroup's LDS (four-step form) and
// the 2D / 3D complex and centered Hermitian convolutions (Secs. 3.1-3.4).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/impconv.h"
#include "runtime.hpp"

namespace impconv {

// Creates, on the current device, what a 1D convolution of these parameters
// would otherwise create on its first call (the three-pass form's column
// twiddle table), so that later calls launch kernels only.
impconv_status conv1d_prepare(int kind, int dt, int64_t batch, int64_t M, int64_t m, uint32_t flags);

// Complex 1D convolution of length m > kRowMax (next_pow2(m) <= 2^17).
impconv_status large1d_plan(int dt, int64_t batch, int64_t M, int64_t m, size_t* work);
impconv_status large1d_run(const DevTables& tb, int dt, int64_t batch, int64_t M, int64_t m,
                           const void* f, const void* g, void* h, void* work, uint32_t flags,
                           hipStream_t s);

// Four-step passes for a ragged size class: count pairs of FFT size N, pair j
// at element d_off[j] with length d_m[j] (device arrays), M = 1.  n2 is the
// column length of the split N = N1 x N2 (0: the default split).
impconv_status large1d_run_ragged(const DevTables& tb, int dt, int64_t count, int64_t N, int64_t maxm,
                                  const void* f, const void* g, void* h, void* work,
                                  const int64_t* d_off, const int64_t* d_m, uint32_t flags,
                                  hipStream_t s, int64_t n2 = 0);

// Default split of a four-step length N into N1 (row, contiguous) x N2
// (column): N2 = 2^floor(log2(N) / 2).
void fourstep_split(int64_t N, int64_t* N1, int64_t* N2);
// Every column length N2 the kernels support for length N (16 <= N2 <=
// 4096, 16 <= N1 <= 8192): the candidates of the autotuner.
std::vector<int64_t> fourstep_splits(int64_t N);

}  // namespace impconv
