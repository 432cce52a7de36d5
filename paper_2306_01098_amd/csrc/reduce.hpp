// Deterministic grid reductions: wave64 shuffles -> LDS -> one partial per
// block -> the last block to finish sums the partials in block order.
#pragma once

#include "common.hpp"

namespace hisq {

// Sum NV doubles over the block.  Result valid in thread 0.  `lds` must hold
// (blockDim.x / 64) * NV doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k)
        v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            lds[wave * NV + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < nwaves; ++w)
                s += lds[w * NV + k];
            v[k] = s;
        }
    }
}

// Thread 0 of every block stores its partials (partials[slot * nblk + blk] for
// slot = slot0 .. slot0+nv-1), then counts the block in *counter.  Returns
// true, in every thread of the block, iff this block finished last; the
// counter is then reset to zero for the next launch.  After a true return all
// partials of all blocks are visible to the block.
__device__ __forceinline__ bool publish_and_check_last(const double *vals, int nv, double *partials,
                                                       int slot0, int blk, int nblk,
                                                       unsigned *counter, unsigned nblocks_total,
                                                       int *lds_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < nv; ++k)
            partials[(size_t)(slot0 + k) * nblk + blk] = vals[k];
        const unsigned prev =
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        const int last = prev == nblocks_total - 1;
        if (last)
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *lds_flag = last;
    }
    __syncthreads();
    const bool last = *lds_flag != 0;
    if (last)
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
    return last;
}

// In the last block (all threads): tot[s] = sum_b partials[s * nblk + b] for
// s < nslots.  Thread t sums the partials t, t + blockDim, ... in order, then
// the block sums the threads in a fixed tree: the result is deterministic.
__device__ __forceinline__ void sum_partials_block(const double *partials, int nslots, int nblk,
                                                   double *tot, int stride = 1) {
    __shared__ double lds[4];
    for (int s = 0; s < nslots; ++s) {
        double v[1] = {0.0};
        const double *p = partials + (size_t)s * nblk;
        for (int b = threadIdx.x; b < nblk; b += blockDim.x)
            v[0] += __builtin_nontemporal_load(p + b);
        block_sum<1>(v, lds);
        if (threadIdx.x == 0)
            tot[(size_t)s * stride] = v[0];
        __syncthreads();
    }
}

}  // namespace hisq
