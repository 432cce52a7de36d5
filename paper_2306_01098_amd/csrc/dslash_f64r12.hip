// Dslash instantiations: links HISQ_FP64R12 (rows 0 and 1 stored), fields HISQ_FP64.
#include "dslash_dispatch.hpp"

namespace hisq {

hipError_t dslash_launch_f64r12(const DslashParams &prm, int epi, DslashShape s, hipStream_t st) {
    return dslash_launch_pair<HISQ_FP64R12, HISQ_FP64>(prm, epi, s, st);
}

}  // namespace hisq
