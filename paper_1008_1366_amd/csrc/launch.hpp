// launch.hpp -- host launchers of the kernel families (one translation unit
// per family so the template instantiations compile in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include "rowconv.hpp"

namespace impconv {

// Largest FFT size of the fused row kernels (LDS-resident, 8192 complex
// values = 64 KB complex64 / 128 KB complex128 plus padding).
constexpr int kRowMax = 8192;

// dt: 0 = complex64, 1 = complex128.  N / NC / NN: FFT size (power of two).
hipError_t launch_row_complex(int dt, int N, const RowArgs& a, hipStream_t s);
hipError_t launch_row_cyclic(int dt, int N, const RowArgs& a, hipStream_t s);
// complex64 with compensated twiddle products (a.flags & kComp, a.twlo set)
hipError_t launch_row_complex_comp(int N, const RowArgs& a, hipStream_t s);
hipError_t launch_row_hermitian(int dt, int NC, const RowArgs& a, hipStream_t s);
hipError_t launch_row_ternary(int dt, int NN, const RowArgs& a, hipStream_t s);
// Whether the ternary row kernel of size NN accumulates its result in h
// residue by residue (rows too long for registers); otherwise each row is
// read completely before any of its outputs is written, so h may be f.
bool row_ternary_accumulates(int dt, int NN);
hipError_t launch_row_realcyclic(int dt, int NC, const RowArgs& a, hipStream_t s);
// General p/q rule: block size NP <= kPqMax (power of two), P in {2, 3};
// a.q residues, a.twq = zeta_{q NP} table.
constexpr int kPqMax = 4096;  // complex64; complex128: kPqMax / 2 (register budget)
constexpr int kPqMaxP = 3;
hipError_t launch_row_pq(int dt, int NP, int P, const RowArgs& a, hipStream_t s);

// Ragged batches: one persistent launch over a work queue of the fused size
// classes (queue.hpp).  d_cls: ncls class records in device memory, ctr: a
// counter in device memory (cleared by the launch), grid: workgroups.
struct QueueClass;
hipError_t launch_row_queue(int dt, const RowArgs& a, const QueueClass* d_cls, int ncls, unsigned* ctr, int grid,
                            hipStream_t s);
// Whether the queue kernel runs FFT size N with E values per thread (the
// row kernels' choice or half of it), and the row kernels' choice.
bool queue_supports(int dt, int N, int E);
int queue_default_E(int dt, int N);

// dst[r][j] = j < copy ? src[r][j] : 0, j < dst_ld
hipError_t launch_pad_rows(int dt, const void* src, void* dst, int64_t nrows, int64_t src_ld,
                           int64_t copy, int64_t dst_ld, hipStream_t s);

// 2D copy with zero fill (see k_copy2d)
hipError_t launch_copy2d(int dt, const void* src, void* dst, int64_t nb, int64_t nsub, int64_t sbs,
                         int64_t sbs2, int64_t sld, int64_t dbs, int64_t dbs2, int64_t dld, int64_t cx,
                         int64_t cy, int64_t dx, int64_t dy, hipStream_t s);

// Column passes (colpass.hpp); N <= kColMax, except, in complex64, the
// ternary passes (N <= 8192: tconv2 with m_x up to 4096, tiles of two
// columns) and the plain FFT pass of the comparators (N <= 16384, tiles of
// one column).  Indexed by dtype.
constexpr int kColMax = 4096;
constexpr int kTerColMax[2] = {8192, 4096};
constexpr int kFftColMax[2] = {16384, 4096};
struct ColArgs;
hipError_t launch_col(int dt, int N, int mode, int dir, const ColArgs& a, hipStream_t s);
hipError_t launch_col_pad(int dt, int N, int mode, const ColArgs& a, hipStream_t s);
// complex64 kPadBwd / kPadFwd with compensated twiddle products (a.twlo set)
hipError_t launch_col_pad_comp(int N, int mode, const ColArgs& a, hipStream_t s);
hipError_t launch_col_cen(int dt, int N, int mode, const ColArgs& a, hipStream_t s);
hipError_t launch_col_ter(int dt, int N, int mode, const ColArgs& a, hipStream_t s);
hipError_t launch_col_fft(int dt, int N, int dir, const ColArgs& a, hipStream_t s);
hipError_t launch_col_fs(int dt, int N, int mode, const ColArgs& a, hipStream_t s);

}  // namespace impconv

#define IMPCONV_POW2_CASES(X) \
    X(1) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192)
#define IMPCONV_COL_CASES(X) \
    X(1) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)
