// Dslash instantiations: links HISQ_FP32R12 (rows 0 and 1 stored), fields HISQ_FP32.
#include "dslash_dispatch.hpp"

namespace hisq {

hipError_t dslash_launch_f32r12(const DslashParams &prm, int epi, DslashShape s, hipStream_t st) {
    return dslash_launch_pair<HISQ_FP32R12, HISQ_FP32>(prm, epi, s, st);
}

}  // namespace hisq
