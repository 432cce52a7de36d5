// Host dispatch of the Dslash over precisions and launch shapes.
#include "internal.hpp"
#include "dslash.hpp"

namespace hisq {

hipError_t dslash_launch_f64(const DslashParams &, int, DslashShape, hipStream_t);
hipError_t dslash_launch_f32(const DslashParams &, int, DslashShape, hipStream_t);
hipError_t dslash_launch_f16(const DslashParams &, int, DslashShape, hipStream_t);
hipError_t dslash_launch_f16f32(const DslashParams &, int, DslashShape, hipStream_t);
hipError_t dslash_launch_f64r12(const DslashParams &, int, DslashShape, hipStream_t);
hipError_t dslash_launch_f32r12(const DslashParams &, int, DslashShape, hipStream_t);
hipError_t dslash_launch_f64w14(const DslashParams &, int, DslashShape, hipStream_t);
hipError_t dslash_launch_f32w14(const DslashParams &, int, DslashShape, hipStream_t);

bool dslash_shape_supported(DslashShape s) {
    const bool var_ok = s.variant == VAR_SITE || s.variant == VAR_DIR || s.variant == VAR_LDS ||
                        (s.variant == VAR_HOP && s.nin <= 2);
    const bool nin_ok = s.nin == 1 || s.nin == 2 || s.nin == 4 || s.nin == 8;
    const bool blk_ok = s.block == 64 || s.block == 128 || s.block == 256 || s.variant == VAR_LDS;
    const bool remap_ok = s.xcd_remap == 0 || s.xcd_remap == 1 || s.xcd_remap == 2;
    return var_ok && nin_ok && blk_ok && remap_ok;
}

bool dslash_shape_fits(DslashShape s, const Geom &g) {
    if (s.variant == VAR_LDS)  // whole pieces of LDS_BAND rows, full wavefronts, the staging within 64 KiB
        return g.nz % 8 == 0 && g.ny % LDS_BAND == 0 && (LDS_BAND * g.hx) % 64 == 0 && LDS_BAND * g.hx <= 256;
    return s.xcd_remap != 2 || g.nz % 8 == 0;
}

bool dslash_shape_fits(DslashShape s, const Geom &g, int fp) {
    if (!dslash_shape_fits(s, g))
        return false;
    return s.variant != VAR_LDS ||
           ((fp == HISQ_FP64 || fp == HISQ_FP32) && lds_stage_bytes(g, fp, s.nin) <= 65536);
}

int dslash_partial_blocks(const Geom &g, DslashShape s) {
    if (s.variant == VAR_LDS)
        return g.vh / (LDS_BAND * g.hx);
    const int sites_per_block = s.variant == VAR_DIR ? s.block / 4 : s.variant == VAR_HOP ? s.block / 16 : s.block;
    return (g.vh + sites_per_block - 1) / sites_per_block;
}

hipError_t launch_dslash(const DslashParams &prm, int lp, int fp, int epi, DslashShape s, hipStream_t st) {
    if (!dslash_shape_supported(s))
        return hipErrorInvalidValue;
    if (s.variant == VAR_LDS && !dslash_shape_fits(s, prm.g, fp))
        s = DslashShape{VAR_SITE, s.nin, 64, prm.g.nz % 8 == 0 ? 2 : 1};  // geometry or format not staged
    if (!dslash_shape_fits(s, prm.g))
        s.xcd_remap = 1;  // z-slab order needs N_z divisible by 8
    if (fp == HISQ_FP32 && prm.nrhs < 2)
        s.nin = 1;  // a one-column FP32 field has no column pairs to load together
    if (lp == HISQ_FP64 && fp == HISQ_FP64)
        return dslash_launch_f64(prm, epi, s, st);
    if (lp == HISQ_FP32 && fp == HISQ_FP32)
        return dslash_launch_f32(prm, epi, s, st);
    if (lp == HISQ_FP16N && fp == HISQ_FP16N)
        return dslash_launch_f16(prm, epi, s, st);
    if (lp == HISQ_FP16N && fp == HISQ_FP32)
        return dslash_launch_f16f32(prm, epi, s, st);
    if (lp == HISQ_FP64R12 && fp == HISQ_FP64)
        return dslash_launch_f64r12(prm, epi, s, st);
    if (lp == HISQ_FP32R12 && fp == HISQ_FP32)
        return dslash_launch_f32r12(prm, epi, s, st);
    if (lp == HISQ_FP64W14 && fp == HISQ_FP64)
        return dslash_launch_f64w14(prm, epi, s, st);
    if (lp == HISQ_FP32W14 && fp == HISQ_FP32)
        return dslash_launch_f32w14(prm, epi, s, st);
    return hipErrorInvalidValue;
}

}  // namespace hisq
