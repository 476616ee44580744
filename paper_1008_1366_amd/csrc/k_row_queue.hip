// Launch unit of the persistent work-queue kernel of ragged batches.
#include "launch.hpp"
#include "queue.hpp"
#include "runtime.hpp"

namespace impconv {

// Clears the queue's counter (a kernel rather than a memset, so that a
// captured graph holds only kernel nodes).
__global__ void k_queue_reset(unsigned* ctr)
{
    if (threadIdx.x == 0) ctr[0] = 0u;
}

hipError_t launch_row_queue(int dt, const RowArgs& a, const QueueClass* d_cls, int ncls, unsigned* ctr, int grid,
                            hipStream_t s)
{
    if (ncls < 1 || ncls > kQueueMaxClasses || grid < 1) return hipErrorInvalidValue;
    timing_begin(s);
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, ctr);
    if (dt)
        hipLaunchKernelGGL(k_ragged_queue<double>, dim3(grid), dim3(kQueueBlock), 0, s, a, d_cls, ncls, ctr);
    else
        hipLaunchKernelGGL(k_ragged_queue<float>, dim3(grid), dim3(kQueueBlock), 0, s, a, d_cls, ncls, ctr);
    timing_end("k_ragged_queue", s);
    return hipGetLastError();
}

bool queue_supports(int dt, int N, int E)
{
    if (N > kRowMax || !queue_fits(N, E)) return false;
    const int e0 = dt ? fft_E<double>(N) : fft_E<float>(N);
    return E == e0 || E == e0 / 2;
}

int queue_default_E(int dt, int N) { return dt ? fft_E<double>(N) : fft_E<float>(N); }

}  // namespace impconv
