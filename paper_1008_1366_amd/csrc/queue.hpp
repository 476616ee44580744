// queue.hpp -- one persistent launch for the fused size classes of a ragged
// batch of complex 1D convolutions (Sec. 2.1 per pair).
//
// The pairs of a size class (FFT size N = 2^ceil(log2 m) <= 8192) are cut
// into items of as many pairs as fill one workgroup of kQueueBlock threads
// (G = N / E threads per pair, E values per thread).  Items are numbered
// class by class, longest N first, so that the items taken first are the
// most expensive ones.  Every workgroup takes the next item number from an
// atomic counter and convolves its pairs with the fused row code of
// k_conv1d_complex (residue split, both transforms, products, forward
// transforms, recombination in registers and LDS), until the numbers run
// out.  The grid holds at most one workgroup per compute unit at a time
// (the exchange buffers of a 512-thread workgroup take 139 KB of LDS), so
// the launch stays resident while the queue drains.
//
// The class table lives in device memory (dynamic indexing of an array in
// the kernel arguments would copy them to scratch); the counter lives in
// the caller's work memory and is cleared by a one-thread kernel before
// each launch (launch_row_queue).
#pragma once
#include "rowconv.hpp"

namespace impconv {

constexpr int kQueueBlock = 512;
constexpr int kQueueMaxClasses = 14;  // N = 1, 2, 4, ..., 8192
#define IMPCONV_QUEUE_CASES(X) \
    X(1) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192)

struct QueueClass {
    const int64_t* off;  // element offsets of the class's pairs (device)
    const int64_t* m;    // their lengths
    int64_t count;       // pairs
    int64_t maxm;        // longest pair
    int64_t item_end;    // items of this class and of every class before it
    int32_t N;           // FFT size
    int32_t E;           // values per thread
};

// Whether a class of FFT size N can run E values per thread in the queue:
// at least radix 2 per stage (unless N = 1), G = N / E threads per pair
// within one workgroup, E dividing N.
__host__ __device__ constexpr bool queue_fits(int N, int E)
{
    return E >= 1 && E <= N && N % E == 0 && (E >= 2 || N == 1) && N / E <= kQueueBlock;
}
// Pairs per item.
__host__ __device__ constexpr int queue_pairs(int N, int E) { return kQueueBlock / (N / E); }
// Complex values of LDS a workgroup needs: two exchange buffers per pair.
template <typename T>
__host__ __device__ constexpr int queue_lds()
{
    return 2 * kQueueBlock * fft_E<T>(8192) + 2 * kQueueBlock * fft_E<T>(8192) / 16;
}

template <typename T, int N, int E>
__device__ __forceinline__ void queue_item(RowArgs a, const QueueClass& k, int64_t j, C<T>* sh, int tid)
{
    constexpr int G = N / E, GQ = kQueueBlock / G;
    constexpr int LDSN = N > E ? lpad_size(N) : 1;
    static_assert(2 * GQ * LDSN <= queue_lds<T>(), "queue exchange buffers exceed the workgroup's LDS");
    const int grp = tid / G, t = tid % G;
    a.row_off = k.off;
    a.row_m = k.m;
    a.nrows = k.count;
    a.m = k.maxm;
    const RowCtx c = row_ctx(a, j * GQ + grp);
    conv_complex_row<T, N, E, true, false>(a, c, t, sh + grp * LDSN, sh + (GQ + grp) * LDSN,
                                           tw_src<T, false>(a, tw_off(N)), tw_src<T, false>(a, tw_off(2 * N)));
}

// Item j of class k: dispatch on (N, E), uniform over the workgroup.
template <typename T, int N>
__device__ __forceinline__ void queue_item_n(const RowArgs& a, const QueueClass& k, int64_t j, C<T>* sh, int tid)
{
    constexpr int E0 = fft_E<T>(N), E1 = fft_E<T>(N) / 2;
    if constexpr (queue_fits(N, E1)) {
        if (k.E == E1) {
            queue_item<T, N, E1>(a, k, j, sh, tid);
            return;
        }
    }
    if constexpr (queue_fits(N, E0)) queue_item<T, N, E0>(a, k, j, sh, tid);
}

template <typename T>
__global__ void __launch_bounds__(kQueueBlock, 2)
k_ragged_queue(RowArgs a, const QueueClass* __restrict__ cls, int ncls, unsigned* ctr)
{
    __shared__ C<T> sh[queue_lds<T>()];
    __shared__ unsigned s_item;
    const int64_t nitems = cls[ncls - 1].item_end;
    int c = 0;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(ctr, 1u);
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();  // every wave has read s_item (and left the last item's LDS) before it changes
        if (item >= nitems) return;
        while (item >= cls[c].item_end) ++c;  // a workgroup's items increase, so c only advances
        const QueueClass k = cls[c];
        const int64_t j = item - (c ? cls[c - 1].item_end : 0);
        // The thread index passes through an empty asm statement on every
        // item, so that no address derived from it is computed once before
        // the loop: each (N, E) variant would keep its own set live across
        // the whole loop and together they would exhaust the registers.
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        switch (k.N) {
#define IMPCONV_QCASE(n) \
    case n: queue_item_n<T, n>(a, k, j, sh, tid); break;
            IMPCONV_QUEUE_CASES(IMPCONV_QCASE)
#undef IMPCONV_QCASE
            default: break;
        }
    }
}

}  // namespace impconv
