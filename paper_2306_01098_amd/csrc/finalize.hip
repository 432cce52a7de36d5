// One-block finalize of a grid reduction: out[s * stride] = sum of the block
// partials of slot s, one wavefront per slot (deterministic).
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

}  // namespace

hipError_t launch_sum_partials(const double *partials, int nslots, int nblk, double *out, int stride,
                               const int *skip, hipStream_t st) {
    sum_partials_kernel<<<1, 1024, 0, st>>>(partials, nslots, nblk, out, stride, skip);
    return hipGetLastError();
}

}  // namespace hisq
