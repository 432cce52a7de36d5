// One-block finalize of a grid reduction: out[s * stride] = sum of the block
// partials of slot s, one wavefront per slot (deterministic); and the
// streaming copy and read used as bandwidth references.
#include "internal.hpp"
#include "reduce.hpp"

namespace hisq {

namespace {

__global__ void __launch_bounds__(1024) sum_partials_kernel(const double *partials, int nslots, int nblk,
                                                           double *out, int stride, const int *skip) {
    if (skip && *skip)
        return;
    sum_partials_block(partials, nslots, nblk, out, stride);
}

// Each block moves 4 x 256 chunks of 16 bytes; thread t takes chunks
// t, t + 256, t + 512, t + 768 of its block's range (coalesced), all four
// loads issued before the stores.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) stream_copy_kernel(const u32x4 *src, u32x4 *dst, size_t n16) {
    const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k * 256 < n16)
            v[k] = __builtin_nontemporal_load(src + base + k * 256);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k * 256 < n16)
            __builtin_nontemporal_store(v[k], dst + base + k * 256);
}

// Read-only reference: each block reads 4 x 256 chunks of 16 bytes (same
// pattern as the copy) and stores the XOR of its 32-bit words in sink[block],
// so the loads cannot be dropped and the result can be checked.
__global__ void __launch_bounds__(256) stream_read_kernel(const u32x4 *src, size_t n16, unsigned *sink) {
    __shared__ unsigned lds[4];
    const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
    u32x4 acc = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k * 256 < n16)
            acc ^= __builtin_nontemporal_load(src + base + k * 256);
    unsigned v = acc.x ^ acc.y ^ acc.z ^ acc.w;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v ^= __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0)
        lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        sink[blockIdx.x] = lds[0] ^ lds[1] ^ lds[2] ^ lds[3];
}

}  // namespace

size_t stream_read_blocks(size_t n16) { return (n16 + 1023) / 1024; }

hipError_t launch_stream_read(const void *src, size_t n16, unsigned *sink, hipStream_t st) {
    const size_t nblk = stream_read_blocks(n16);
    if (nblk > 0x7fffffffu)
        return hipErrorInvalidValue;
    stream_read_kernel<<<dim3((unsigned)nblk), 256, 0, st>>>(static_cast<const u32x4 *>(src), n16, sink);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void *src, void *dst, size_t n16, hipStream_t st) {
    const size_t nblk = (n16 + 1023) / 1024;
    if (nblk > 0x7fffffffu)
        return hipErrorInvalidValue;
    stream_copy_kernel<<<dim3((unsigned)nblk), 256, 0, st>>>(static_cast<const u32x4 *>(src),
                                                              static_cast<u32x4 *>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partials, int nslots, int nblk, double *out, int stride,
                               const int *skip, hipStream_t st) {
    sum_partials_kernel<<<1, 1024, 0, st>>>(partials, nslots, nblk, out, stride, skip);
    return hipGetLastError();
}

}  // namespace hisq
