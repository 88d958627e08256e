// md_reduce.h -- fixed-order reductions shared by the force and adjoint kernels.
//
// Each workgroup reduces its threads' partial sums with a fixed butterfly and a
// fixed cross-wave order, writes them to partial[block][4], and the last
// workgroup to finish (device-scope counter) adds all blocks' partials in block
// order.  The result is therefore bitwise repeatable for a given grid size,
// which plays the role of the thread-local energy accumulators of Sec. II.C.
#pragma once

#include "md_internal.h"

namespace mdred {

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sums v[0..3] over a block of up to 512 threads (a multiple of 64); every
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

__device__ __forceinline__ void store_agent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double load_agent(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Writes this block's partial sums; returns true (in every thread) for the
// last block to finish, which then holds every block's partials in v[] summed
// in block order.
__device__ __forceinline__ bool last_block_sum4(double v[4], double *partial, uint32_t *done,
                                                double *lds)
{
    __shared__ int is_last;
    block_sum4(v, lds);
    if (threadIdx.x == 0) {
        for (int c = 0; c < 4; c++) store_agent(&partial[blockIdx.x * 4 + c], v[c]);
        __threadfence();
        const uint32_t prev = atomicAdd(done, 1u);
        is_last = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x)
        for (int c = 0; c < 4; c++) s[c] += load_agent(&partial[b * 4 + c]);
    block_sum4(s, lds);
    for (int c = 0; c < 4; c++) v[c] = s[c];
    if (threadIdx.x == 0) *done = 0u;
    return true;
}

} // namespace mdred
