// Dslash instantiations: links HISQ_FP64, fields HISQ_FP64.
#include "dslash_dispatch.hpp"

namespace hisq {

hipError_t dslash_launch_f64(const DslashParams &prm, int epi, DslashShape s, hipStream_t st) {
    return dslash_launch_pair<HISQ_FP64, HISQ_FP64>(prm, epi, s, st);
}

}  // namespace hisq
