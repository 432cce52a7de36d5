// Deterministic grid reductions: wave64 shuffles -> LDS -> one partial per
// block, stored by the reducing kernel; a one-block finalize kernel launched
// after it sums the partials in block order.  (A "last block finishes"
// scheme needs an agent-scope release per block, which on the multi-XCD
// MI355X writes back the L2 each time and made reducing kernels 3-7x slower.)
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

// The same for the column-pair vector kernels, whose blocks of 2 b threads
// cover the b sites of a b-thread block for two columns: lane l of wave w
// holds site 32 (w & 1) + (l >> 1) of the block's 64-site group w >> 1 for
// column l & 1.  The additions are those of block_sum over the b sites of
// one column, in the same order (the sites 32 apart first, then the
// butterfly over the remaining five site bits, then the 64-site groups in
// order), so a column's partials are bitwise the ones of a one-column block.
// The sum of the even lanes' column is valid in thread 0, of the odd lanes'
// in thread 1.  `lds` must hold (blockDim.x / 128) * 64 * NV doubles.
template <int NV>
__device__ __forceinline__ void block_sum_pair(double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ngroups = blockDim.x >> 7;
    const int g = wave >> 1;
    if (wave & 1) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            lds[(g * 64 + lane) * NV + k] = v[k];
    }
    __syncthreads();
    if (!(wave & 1)) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            v[k] += lds[(g * 64 + lane) * NV + k];
#pragma unroll
            for (int o = 32; o >= 2; o >>= 1)
                v[k] += __shfl_xor(v[k], o, 64);
        }
    }
    __syncthreads();
    if (!(wave & 1) && lane < 2) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            lds[(g * 2 + lane) * NV + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 2) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int q = 0; q < ngroups; ++q)
                s += lds[(q * 2 + threadIdx.x) * NV + k];
            v[k] = s;
        }
    }
}

// Sums of NV values (NV a power of two <= 64) over the wavefront with
// log2(NV) halving exchanges: at offset 32, 16, ... each lane gives the
// partner half of its remaining values and keeps the other half, so NV/2 +
// NV/4 + ... + 1 shuffles replace NV full trees; the remaining offsets finish
// one value per lane.  Afterwards v[0] of lane l holds the total of value
// index wave_multi_index<NV>(l) (the same in every lane of a group of
// 64 / NV).  The order of additions is fixed: deterministic.
template <int NV> __device__ __forceinline__ int wave_multi_index(int lane) {
    int idx = 0;
#pragma unroll
    for (int o = 32, n = NV; n > 1; o >>= 1, n >>= 1)
        idx = 2 * idx + ((lane & o) ? 1 : 0);
    return idx;
}

template <int NV, typename T> __device__ __forceinline__ void wave_sum_multi(T (&v)[NV]) {
    static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two <= 64");
    const int lane = threadIdx.x & 63;
    int o = 32;
#pragma unroll
    for (int n = NV; n > 1; n >>= 1, o >>= 1) {
        const bool upper = (lane & o) != 0;
#pragma unroll
        for (int k = 0; k < n / 2; ++k) {
            const T give = upper ? v[k] : v[k + n / 2];
            const T keep = upper ? v[k + n / 2] : v[k];
            v[k] = keep + __shfl_xor(give, o, 64);
        }
    }
#pragma unroll
    for (; o > 0; o >>= 1)
        v[0] += __shfl_xor(v[0], o, 64);
}

// Sum of one slot by one wavefront: lane l adds partials l, l + 64, l + 128,
// ... in that order (eight loads in flight per step), then the wave adds the
// lanes in a fixed shuffle tree.  The result is the same whichever wave runs
// it, so the sum is deterministic.  Returns the total in every lane.  NT:
// non-temporal loads (one reader); plain loads when every block of a grid
// reads the same slot, so it stays in the L2.
template <bool NT = true> __device__ __forceinline__ double ld_partial(const double *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT = true> __device__ __forceinline__ double wave_sum_slot(const double *p, int nblk) {
    const int lane = threadIdx.x & 63;
    double v = 0.0;
    int b = lane;
    for (; b + 7 * 64 < nblk; b += 8 * 64) {
        double t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            t[k] = ld_partial<NT>(p + b + k * 64);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            v += t[k];
    }
    for (; b < nblk; b += 64)
        v += ld_partial<NT>(p + b);
    return wave_sum(v);
}

// In one block (all threads): tot[s * stride] = sum_b partials[s * nblk + b]
// for s < nslots, slot s summed by wave s mod (blockDim.x / 64).  Ends with a
// block barrier, so `tot` may be shared memory read by the whole block.
__device__ __forceinline__ void sum_partials_block(const double *partials, int nslots, int nblk,
                                                   double *tot, int stride = 1) {
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int s = wave; s < nslots; s += nw) {
        const double v = wave_sum_slot<true>(partials + (size_t)s * nblk, nblk);
        if ((threadIdx.x & 63) == 0)
            tot[(size_t)s * stride] = v;
    }
    __syncthreads();
}

}  // namespace hisq
