// Dslash instantiations: links HISQ_FP16N, fields HISQ_FP16N.
#include "dslash_dispatch.hpp"

namespace hisq {

hipError_t dslash_launch_f16(const DslashParams &prm, int epi, DslashShape s, hipStream_t st) {
    return dslash_launch_pair<HISQ_FP16N, HISQ_FP16N>(prm, epi, s, st);
}

}  // namespace hisq
