// The Dslash autotuner: times every supported launch shape on the caller's
// buffers with HIP events and keeps the fastest per (extents, precisions,
// nrhs) in the context.
#include <algorithm>
#include <vector>

#include "api_util.hpp"
#include "dslash.hpp"

namespace hisq {

// Built-in shapes (measured on MI355X at 32^3x8 and 48^3x12): one thread per
// site (four lanes per site on lattices too small to fill the chip); with
// several right-hand sides one thread per site holding four of them (FP16N
// links: two; FP32 links and fields: eight) in blocks of 256 (FP32 and FP16N
// fields) or 128 (FP64 fields; eight FP32 rhs); FP32 fields of at least four
// columns on lattices the LDS staging fits: the LDS-staged mapping, four rhs
// per thread.
DslashShape default_shape(const Geom &g, int lp, int fp, int nrhs) {
    // measured on 32^3x8 at one right-hand side and 48^3x12 at 4 and 16:
    // the per-site mapping wins everywhere once the N_outer groups of a site
    // range run together; more than 4 (FP16N: 2) accumulators per thread cost
    // more in occupancy than the shared link loads save.  At one right-hand
    // side the z-slab block order (when N_z allows it) keeps the t-hops inside
    // each XCD: 32^3x8 FP64 53.1 -> 48.1 us.
    DslashShape s;
    s.variant = VAR_SITE;
    s.xcd_remap = 1;
    if (nrhs == 1) {
        s.nin = 1;
        // Small lattices cannot fill 256 CUs with one thread per site in
        // blocks of 256: up to 16384 sites per parity (49152 for FP32 and
        // FP16N links) four lanes per site (8^4 .. 16^3x8: 9.6-16.1 -> 9.2-9.3
        // us FP64; 16^4 FP32 12.2 -> 9.4 us), below 131072 blocks of 64
        // (24^3x6 FP64 19.4 -> 16.6 us)
        const bool wide = lp == HISQ_FP64 || lp == HISQ_FP64R12 || lp == HISQ_FP64W14;
        if (g.vh <= (wide ? 16384 : 49152)) {
            s.variant = VAR_DIR;
            // inside the CG graph blocks of 64 spread these lattices over more
            // CUs (8^4 FP64 CG 17.3 -> 15.6 ms; the isolated launch is the same)
            s.block = 64;
            return s;
        }
        if (g.vh < 131072) {
            s.block = 64;
            s.xcd_remap = g.nz % 8 == 0 ? 2 : 1;
            return s;
        }
        if (g.nz % 8 == 0) {
            // FP16N links too: the CG's fused scalar step sums 4x fewer block
            // partials (32^3x8 FP16N-link CG 7.53 -> 7.41 ms; the Dslash alone
            // the same within 1 %)
            s.xcd_remap = 2;
            s.block = 256;
        } else {
            s.block = 128;
        }
        return s;
    }
    // FP32 fields: the x- and y-hop vectors of four rhs per thread staged in
    // LDS where the lattice allows it (16 rhs at 48^3x12: FP32 links 461 ->
    // 421 us, FP32R12 413 -> 365 us; the 16-rhs CG with FP32 links 0.407 ->
    // 0.390 s, FP32R12 0.385 -> 0.360 s, FP16N links 0.408 -> 0.348 s)
    if (fp == HISQ_FP32 && nrhs >= 4) {
        const DslashShape l{VAR_LDS, 4, LDS_BAND * g.hx, 2};
        if (dslash_shape_fits(l, g, fp))
            return l;
    }
    const int cap = lp == HISQ_FP16N ? 2 : 4;
    s.nin = nrhs >= cap ? cap : 2;
    // 16 rhs at 48^3x12, blocks of 64 -> 128: FP32 520 -> 476 us, FP32R12
    // 467 -> 431 us, FP64 995 -> 935 us, FP16N 466 -> 457 us; 128 -> 256 with
    // FP32 fields and FP32-family links: FP32 476-514 -> 473-483 us, FP32R12
    // 430-465 -> 427-433 us over four boxes (FP64 mixed, 935-1001 -> 970-973);
    // FP16N fields 452 -> 433 us
    s.block = (fp == HISQ_FP32 && lp != HISQ_FP16N) || fp == HISQ_FP16N ? 256 : 128;
    // FP32 links and fields, whole groups of 8: eight rhs per thread in blocks
    // of 128 (16 rhs at 48^3x12: 476 -> 460 us; the 16-rhs CG 0.421 -> 0.407
    // s; FP32R12 links gain nothing from it)
    if (lp == HISQ_FP32 && fp == HISQ_FP32 && nrhs % 8 == 0) {
        s.nin = 8;
        s.block = 128;
    }
    // z-slab order in 8-row y-bands: 16 rhs at 48^3x12, FP32 606 -> 585 us,
    // FP64 1231 -> 1105 us
    if (g.nz % 8 == 0)
        s.xcd_remap = 2;
    return s;
}

std::vector<DslashShape> candidate_shapes(const Geom &g, int nrhs, int lp, int fp) {
    std::vector<DslashShape> out;
    // LDS-staged neighbours: one block per piece of rows, block size fixed
    // by N_x, z-slab order
    for (int nin : {1, 2, 4, 8}) {
        const DslashShape s{VAR_LDS, nin, LDS_BAND * g.hx, 2};
        if (nin <= nrhs && dslash_shape_fits(s, g, fp) &&
            !((lp == HISQ_FP64 || lp == HISQ_FP64R12 || lp == HISQ_FP64W14) && nin > 4))
            out.push_back(s);
    }
    for (int var : {VAR_SITE, VAR_DIR, VAR_HOP})
        for (int nin : {1, 2, 4, 8}) {
            if (nin > 1 && nin > nrhs)
                continue;
            if (var == VAR_HOP && nin > 2)
                continue;
            if (var == VAR_SITE && (lp == HISQ_FP64 || lp == HISQ_FP64R12 || lp == HISQ_FP64W14) && nin > 4)
                continue;  // exceeds the register file (spills)
            for (int block : {64, 128, 256})
                for (int remap : {0, 1, 2})
                    if (remap != 2 || g.nz % 8 == 0)
                        out.push_back(DslashShape{var, nin, block, remap});
        }
    return out;
}

// Median time (ms) of `reps` launches of one shape; <0 on a launch error.
static float time_shape(const DslashParams &prm, int lp, int fp, DslashShape s, hipStream_t st, int reps,
                        hipEvent_t e0, hipEvent_t e1, hipError_t *err) {
    std::vector<float> t;
    for (int k = 0; k < 2; ++k) {  // warm-up
        *err = launch_dslash(prm, lp, fp, EPI_PLAIN, s, st);
        if (*err != hipSuccess)
            return -1.f;
    }
    for (int k = 0; k < reps; ++k) {
        hipEventRecord(e0, st);
        *err = launch_dslash(prm, lp, fp, EPI_PLAIN, s, st);
        hipEventRecord(e1, st);
        if (*err != hipSuccess)
            return -1.f;
        *err = hipEventSynchronize(e1);
        if (*err != hipSuccess)
            return -1.f;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

hisq_status tune_dslash(hisq_context *ctx, const Geom &g, int lp, int fp, int nrhs, const void *links,
                        const void *in, void *out, hipStream_t st, DslashShape *best_out) {
    DslashParams prm{};
    prm.g = g;
    prm.out_parity = 0;
    prm.nrhs = nrhs;
    prm.links = static_cast<const char *>(links);
    prm.in = in;
    prm.out = out;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess)
        return device_fail(e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        hipEventDestroy(e0);
        return device_fail(e, "hipEventCreate");
    }
    DslashShape best = default_shape(g, lp, fp, nrhs);
    float best_ms = 1e30f;
    hisq_status status = HISQ_OK;
    for (const DslashShape &s : candidate_shapes(g, nrhs, lp, fp)) {
        hipError_t err = hipSuccess;
        const float ms = time_shape(prm, lp, fp, s, st, 5, e0, e1, &err);
        if (err != hipSuccess) {
            status = device_fail(err, "tune_dslash");
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = s;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (status != HISQ_OK)
        return status;
    ctx->store(g, lp, fp, nrhs, best);
    if (best_out)
        *best_out = best;
    return HISQ_OK;
}

}  // namespace hisq

using namespace hisq;

extern "C" {

hisq_status hisq_tune_dslash(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, int32_t nrhs,
                             const void *links, const void *in, void *out, void *stream) {
    if (!ctx)
        return fail(HISQ_ERR_INVALID_ARG, "ctx is NULL (the tuned shape is kept in the context)");
    hisq_status s = check_lattice(lat);
    if (s == HISQ_OK) s = check_prec(prec);
    if (s == HISQ_OK) s = check_nrhs(nrhs);
    if (s == HISQ_OK) s = check_ptr(links, "links");
    if (s == HISQ_OK) s = check_ptr(in, "in");
    if (s == HISQ_OK) s = check_ptr(out, "out");
    if (s == HISQ_OK && in == out)
        s = fail(HISQ_ERR_INVALID_ARG, "in and out must not alias");
    if (s == HISQ_OK) s = set_device(ctx);
    if (s != HISQ_OK)
        return s;
    return tune_dslash(ctx, make_geom(*lat), prec, field_prec_of(prec), nrhs, links, in, out, static_cast<hipStream_t>(stream),
                       nullptr);
}

hisq_status hisq_get_dslash_shape(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, int32_t nrhs,
                                  hisq_dslash_shape *shape) {
    hisq_status s = check_lattice(lat);
    if (s == HISQ_OK) s = check_prec(prec);
    if (s == HISQ_OK) s = check_nrhs(nrhs);
    if (s == HISQ_OK) s = check_ptr(shape, "shape");
    if (s != HISQ_OK)
        return s;
    const DslashShape d = pick_shape(ctx, make_geom(*lat), prec, field_prec_of(prec), nrhs);
    shape->variant = d.variant;
    shape->nin = d.nin;
    shape->block = d.block;
    shape->xcd_remap = d.xcd_remap;
    return HISQ_OK;
}

hisq_status hisq_set_dslash_shape(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, int32_t nrhs,
                                  const hisq_dslash_shape *shape) {
    if (!ctx)
        return fail(HISQ_ERR_INVALID_ARG, "ctx is NULL");
    hisq_status s = check_lattice(lat);
    if (s == HISQ_OK) s = check_prec(prec);
    if (s == HISQ_OK) s = check_nrhs(nrhs);
    if (s == HISQ_OK) s = check_ptr(shape, "shape");
    if (s != HISQ_OK)
        return s;
    DslashShape d{shape->variant, shape->nin, shape->block, shape->xcd_remap};
    if (d.variant == VAR_LDS) {  // block size and order follow from the lattice
        const Geom g = make_geom(*lat);
        d.block = LDS_BAND * g.hx;
        d.xcd_remap = 2;
        const int fp = prec == HISQ_FP16N ? HISQ_FP32 : field_prec_of(prec);
        if (!dslash_shape_fits(d, g, fp))
            return fail(HISQ_ERR_INVALID_ARG,
                        "the LDS-staged Dslash needs N_z and N_y divisible by 8, N_x in {16, 32, 48, 64}, FP64 or "
                        "FP32 fields and at most 64 KiB of staging for nin = %d",
                        d.nin);
    }
    if (!dslash_shape_supported(d))
        return fail(HISQ_ERR_INVALID_ARG, "unsupported shape (variant %d, nin %d, block %d, remap %d)", d.variant,
                    d.nin, d.block, d.xcd_remap);
    if (!dslash_shape_fits(d, make_geom(*lat)))
        return fail(HISQ_ERR_INVALID_ARG, "block order 2 needs N_z divisible by 8 (N_z = %d)", lat->dims[2]);
    ctx->store(make_geom(*lat), prec, field_prec_of(prec), nrhs, d);
    if (prec == HISQ_FP16N)  // also the FP16-link, FP32-field Dslash inside mixed-precision CG
        ctx->store(make_geom(*lat), prec, HISQ_FP32, nrhs, d);
    return HISQ_OK;
}

}  // extern "C"
