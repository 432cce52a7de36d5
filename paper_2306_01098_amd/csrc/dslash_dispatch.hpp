// Template dispatch of the Dslash kernels over (variant, NIN, epilogue) for
// one (link precision, field precision) pair; each pair is instantiated in
// its own translation unit so the instantiations compile in parallel.
#pragma once

#include "internal.hpp"
#include "dslash.hpp"

namespace hisq {

// Non-temporal link loads: only when each link is read once (one group of
// right-hand sides), the format profits (FP64, FP32, W14) and the link set
// exceeds the MALL, so that ordinary loads would leave nothing cached for the
// next application.
constexpr size_t MALL_BYTES = (size_t)256 << 20;
template <int LP> inline bool links_stream(const Geom &g, int nouter) {
    return LinkIO<LP>::stream && nouter == 1 && links_bytes(g, LP) > MALL_BYTES;
}

template <int LP, int FP, int NIN, int EPI>
hipError_t dslash_go(const DslashParams &prm, DslashShape s, hipStream_t st) {
    if (s.variant == VAR_LDS) {
        // one block per piece of LDS_BAND y-rows at fixed (t, z), in the
        // banded z-slab order (dslash_shape_fits checked the geometry)
        if constexpr (FP == HISQ_FP64 || FP == HISQ_FP32) {
            const int threads = LDS_BAND * prm.g.hx;
            const int nsb = prm.g.vh / threads;
            const int nouter = (prm.nrhs + NIN - 1) / NIN;
            DslashParams p = prm;
            p.xcd_remap = 2;
            p.band = LDS_BAND;
            const size_t shm = lds_stage_bytes(prm.g, FP, NIN);
            const bool nt = links_stream<LP>(prm.g, nouter);
            if (nt)
                dslash_lds_kernel<LP, FP, NIN, EPI, LinkIO<LP>::stream>
                    <<<dim3((unsigned)(nsb * nouter)), threads, shm, st>>>(p);
            else
                dslash_lds_kernel<LP, FP, NIN, EPI, false><<<dim3((unsigned)(nsb * nouter)), threads, shm, st>>>(p);
            hipError_t e = hipGetLastError();
            if (e == hipSuccess && EPI == EPI_AXPY_DOT && p.dot_out != nullptr)
                e = launch_sum_partials(p.partials, p.nrhs, nsb, p.dot_out, p.dot_stride > 0 ? p.dot_stride : 1,
                                        p.skip, st);
            return e;
        } else {
            return hipErrorInvalidValue;
        }
    }
    const int sites_per_block = s.variant == VAR_DIR ? s.block / 4 : s.variant == VAR_HOP ? s.block / 16 : s.block;
    const int nsb = (prm.g.vh + sites_per_block - 1) / sites_per_block;
    const int nouter = (prm.nrhs + NIN - 1) / NIN;
    const dim3 grid((unsigned)(nsb * nouter));
    DslashParams p = prm;
    p.xcd_remap = s.xcd_remap;
    p.band = zslab_band(prm.g, prm.nrhs);
    const bool nt = links_stream<LP>(prm.g, nouter);
    if (s.variant == VAR_HOP) {
        if constexpr (NIN <= 2) {
            if (nt)
                dslash_hop_kernel<LP, FP, NIN, EPI, LinkIO<LP>::stream><<<grid, s.block, 0, st>>>(p);
            else
                dslash_hop_kernel<LP, FP, NIN, EPI, false><<<grid, s.block, 0, st>>>(p);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (s.variant == VAR_DIR) {
        if (nt)
            dslash_dir_kernel<LP, FP, NIN, EPI, LinkIO<LP>::stream><<<grid, s.block, 0, st>>>(p);
        else
            dslash_dir_kernel<LP, FP, NIN, EPI, false><<<grid, s.block, 0, st>>>(p);
    } else {
        if (nt)
            dslash_site_kernel<LP, FP, NIN, EPI, LinkIO<LP>::stream><<<grid, s.block, 0, st>>>(p);
        else
            dslash_site_kernel<LP, FP, NIN, EPI, false><<<grid, s.block, 0, st>>>(p);
    }
    hipError_t e = hipGetLastError();
    // dot_out == nullptr: the caller sums the partials itself
    if (e == hipSuccess && EPI == EPI_AXPY_DOT && p.dot_out != nullptr)
        e = launch_sum_partials(p.partials, p.nrhs, nsb, p.dot_out, p.dot_stride > 0 ? p.dot_stride : 1, p.skip,
                                st);
    return e;
}

template <int LP, int FP, int EPI>
hipError_t dslash_by_nin(const DslashParams &prm, DslashShape s, hipStream_t st) {
    switch (s.nin) {
    case 1: return dslash_go<LP, FP, 1, EPI>(prm, s, st);
    case 2: return dslash_go<LP, FP, 2, EPI>(prm, s, st);
    case 4: return dslash_go<LP, FP, 4, EPI>(prm, s, st);
    case 8: return dslash_go<LP, FP, 8, EPI>(prm, s, st);
    default: return hipErrorInvalidValue;
    }
}

template <int LP, int FP>
hipError_t dslash_launch_pair(const DslashParams &prm, int epi, DslashShape s, hipStream_t st) {
    switch (epi) {
    case EPI_PLAIN: return dslash_by_nin<LP, FP, EPI_PLAIN>(prm, s, st);
    case EPI_AXPY: return dslash_by_nin<LP, FP, EPI_AXPY>(prm, s, st);
    case EPI_AXPY_DOT: return dslash_by_nin<LP, FP, EPI_AXPY_DOT>(prm, s, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hisq
