// md_reduce.h -- fixed-order reductions shared by the force and adjoint kernels.
//
// Each workgroup reduces its threads' partial sums with a fixed butterfly and a
// fixed cross-wave order and writes them to partial[block][4]; a one-workgroup
// launch that follows the producing launch on its stream adds all blocks'
// partials in block order (the launch boundary orders the two, so no
// workgroup waits on a device-wide fence).  The result is therefore bitwise
// repeatable for a given grid size, which plays the role of the thread-local
// energy accumulators of Sec. II.C.
#pragma once

#include "md_internal.h"

namespace mdred {

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sums v[0..3] over a block of up to 1024 threads (a multiple of 64); every
// thread receives the totals, added wave by wave in wave order
__device__ __forceinline__ void block_sum4(double v[4], double *lds /* [4 * waves] */)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = (int)(blockDim.x >> 6);
    for (int c = 0; c < 4; c++) v[c] = wave_sum(v[c]);
    __syncthreads();
    if (lane == 0)
        for (int c = 0; c < 4; c++) lds[w * 4 + c] = v[c];
    __syncthreads();
    for (int c = 0; c < 4; c++) {
        double t = lds[c];
        for (int k = 1; k < nw; k++) t += lds[4 * k + c];
        v[c] = t;
    }
    __syncthreads();
}

// Writes this block's totals of v[0..3] to partial[block][4] (every thread
// receives the totals in v).
__device__ __forceinline__ void block_to_partial4(double v[4], double *partial, double *lds)
{
    block_sum4(v, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; c++) partial[blockIdx.x * 4 + c] = v[c];
}

// The totals of the partials of g blocks, added in block order: thread t takes
// blocks t, t + T, ..., then the block sums its threads as block_sum4 does
// (every thread receives the totals in v).
__device__ __forceinline__ void sum_partials4(const double *partial, int32_t g, double v[4], double *lds)
{
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t b = threadIdx.x; b < g; b += blockDim.x)
        for (int c = 0; c < 4; c++) s[c] += partial[b * 4 + c];
    block_sum4(s, lds);
    for (int c = 0; c < 4; c++) v[c] = s[c];
}

} // namespace mdred
