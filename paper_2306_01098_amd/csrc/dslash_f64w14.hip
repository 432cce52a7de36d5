// Dslash instantiations: links HISQ_FP64W14 (fat links in full, Naik links in 14 reals), fields HISQ_FP64.
#include "dslash_dispatch.hpp"

namespace hisq {

hipError_t dslash_launch_f64w14(const DslashParams &prm, int epi, DslashShape s, hipStream_t st) {
    return dslash_launch_pair<HISQ_FP64W14, HISQ_FP64>(prm, epi, s, st);
}

}  // namespace hisq
