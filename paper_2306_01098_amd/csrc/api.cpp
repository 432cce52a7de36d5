// C ABI entry points: argument validation (host only, before any HIP call),
// error reporting and dispatch to the kernels.
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "api_util.hpp"
#include "dslash.hpp"

using namespace hisq;

namespace hisq {

thread_local std::string g_last_error;

hisq_status fail(hisq_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

hisq_status device_fail(hipError_t e, const char *where) {
    return fail(HISQ_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

hisq_status check_lattice(const hisq_lattice *lat) {
    if (!lat)
        return fail(HISQ_ERR_INVALID_ARG, "lattice descriptor is NULL");
    int64_t v = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const int n = lat->dims[mu];
        if (n < 4 || (n & 1))
            return fail(HISQ_ERR_INVALID_ARG, "extent dims[%d] = %d must be even and >= 4", mu, n);
        v *= n;
    }
    if (v > (int64_t)1 << 30)
        return fail(HISQ_ERR_INVALID_ARG, "lattice volume %lld exceeds 2^30 sites", (long long)v);
    if (lat->t_bc != 1 && lat->t_bc != -1)
        return fail(HISQ_ERR_INVALID_ARG, "t_bc = %d must be +1 or -1", lat->t_bc);
    return HISQ_OK;
}

hisq_status check_prec(int prec) {
    if (prec != HISQ_FP64 && prec != HISQ_FP32 && prec != HISQ_FP16N && prec != HISQ_FP64R12 &&
        prec != HISQ_FP32R12 && prec != HISQ_FP64W14 && prec != HISQ_FP32W14)
        return fail(HISQ_ERR_INVALID_ARG, "unknown precision %d", prec);
    return HISQ_OK;
}

hisq_status check_nrhs(int nrhs) {
    if (nrhs < 1 || nrhs > HISQ_MAX_RHS)
        return fail(HISQ_ERR_INVALID_ARG, "nrhs = %d outside [1, %d]", nrhs, HISQ_MAX_RHS);
    return HISQ_OK;
}

hisq_status check_ptr(const void *p, const char *name) {
    if (!p)
        return fail(HISQ_ERR_INVALID_ARG, "%s is NULL", name);
    return HISQ_OK;
}

hisq_status set_device(hisq_context *ctx) {
    if (!ctx)
        return HISQ_OK;
    const hipError_t e = hipSetDevice(ctx->device);
    return e == hipSuccess ? HISQ_OK : device_fail(e, "hipSetDevice");
}

size_t apply_m_dot_partials_max(const Geom &g, int nrhs) {
    // the smallest site block of any launch shape is 4 sites (sixteen lanes
    // per site in blocks of 64 threads)
    return (size_t)nrhs * (size_t)((g.vh + 3) / 4);
}

hisq_status check_apply_m_dot(hisq_context *ctx, const hisq_lattice *lat, int link_prec, int field_prec, double mass,
                              const void *links, const void *in_even, void *out_even, void *tmp_odd, int nrhs,
                              double *dot_out, ApplyMDot *a) {
    TRY(check_lattice(lat));
    TRY(check_prec(link_prec));
    TRY(check_prec(field_prec));
    TRY(check_nrhs(nrhs));
    const int fp = field_prec_of(field_prec);
    if (fp != field_prec_of(link_prec) && !(link_prec == HISQ_FP16N && fp == HISQ_FP32))
        return fail(HISQ_ERR_INVALID_ARG, "no operator with links of precision %d and fields of precision %d",
                    link_prec, field_prec);
    TRY(check_ptr(links, "links"));
    TRY(check_ptr(in_even, "in_even"));
    TRY(check_ptr(out_even, "out_even"));
    TRY(check_ptr(tmp_odd, "tmp_odd"));
    TRY(check_ptr(dot_out, "dot_out"));
    if (in_even == out_even || tmp_odd == in_even || tmp_odd == out_even)
        return fail(HISQ_ERR_INVALID_ARG, "in_even, out_even and tmp_odd must be distinct");
    if (!(mass == mass) || mass * mass <= 0.0 || mass * mass > 1e300)
        return fail(HISQ_ERR_INVALID_ARG, "mass^2 must be positive and finite (mass = %g)", mass);
    a->g = make_geom(*lat);
    a->lp = link_prec;
    a->fp = fp;
    a->mass = mass;
    a->links = static_cast<const char *>(links);
    a->in = in_even;
    a->out = out_even;
    a->tmp = tmp_odd;
    a->nrhs = nrhs;
    a->dot = dot_out;
    a->shape = pick_shape(ctx, a->g, link_prec, fp, nrhs);
    a->partials = (size_t)nrhs * dslash_partial_blocks(a->g, a->shape);
    return HISQ_OK;
}

// D_oe in -> tmp, then out = m^2 in - D_eo tmp with the block partials of
// Re <in, out> in `partials` and their fixed-order sum in dot[0..nrhs).
hisq_status run_apply_m_dot(const ApplyMDot &a, double *partials, hipStream_t st) {
    DslashParams prm{};
    prm.g = a.g;
    prm.nrhs = a.nrhs;
    prm.links = a.links;
    prm.out_parity = 1;
    prm.in = a.in;
    prm.out = a.tmp;
    hipError_t e = launch_dslash(prm, a.lp, a.fp, EPI_PLAIN, a.shape, st);
    if (e != hipSuccess)
        return device_fail(e, "apply_m_dot (D_oe)");
    prm.out_parity = 0;
    prm.in = a.tmp;
    prm.out = a.out;
    prm.y = a.in;
    prm.ad = -1.0;
    prm.ay = a.mass * a.mass;
    prm.partials = partials;
    prm.dot_out = a.dot;
    prm.dot_stride = 1;
    e = launch_dslash(prm, a.lp, a.fp, EPI_AXPY_DOT, a.shape, st);
    return e == hipSuccess ? HISQ_OK : device_fail(e, "apply_m_dot (D_eo)");
}

DslashShape pick_shape(hisq_context *ctx, const Geom &g, int lp, int fp, int nrhs) {
    if (ctx) {
        DslashShape s;
        if (ctx->lookup(g, lp, fp, nrhs, &s))
            return s;
    }
    return default_shape(g, lp, fp, nrhs);
}

}  // namespace hisq


extern "C" {

hisq_status hisq_context_create(hisq_context **ctx, int32_t device) {
    if (!ctx)
        return fail(HISQ_ERR_INVALID_ARG, "ctx is NULL");
    *ctx = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess)
        return device_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n)
        return fail(HISQ_ERR_INVALID_ARG, "device %d outside [0, %d)", device, n);
    hisq_context *c = new (std::nothrow) hisq_context();
    if (!c)
        return fail(HISQ_ERR_DEVICE, "out of host memory");
    c->device = device;
    const hisq_status s = noalloc_scratch_setup(device);
    if (s != HISQ_OK) {
        delete c;
        return s;
    }
    *ctx = c;
    return HISQ_OK;
}

void hisq_context_destroy(hisq_context *ctx) { delete ctx; }

const char *hisq_status_string(hisq_status s) {
    switch (s) {
    case HISQ_OK: return "ok";
    case HISQ_ERR_INVALID_ARG: return "invalid argument";
    case HISQ_ERR_NOT_CONVERGED: return "not converged";
    case HISQ_ERR_BREAKDOWN: return "breakdown";
    case HISQ_ERR_DEVICE: return "device error";
    case HISQ_ERR_WORKSPACE: return "workspace too small";
    case HISQ_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *hisq_last_error(void) { return g_last_error.c_str(); }

size_t hisq_links_bytes(const hisq_lattice *lat, hisq_prec prec) {
    if (check_lattice(lat) != HISQ_OK || check_prec(prec) != HISQ_OK)
        return 0;
    const Geom g = make_geom(*lat);
    return links_bytes(g, prec);
}

size_t hisq_field_bytes(const hisq_lattice *lat, hisq_prec prec, int32_t nrhs) {
    if (check_lattice(lat) != HISQ_OK || check_prec(prec) != HISQ_OK || check_nrhs(nrhs) != HISQ_OK)
        return 0;
    return field_bytes(make_geom(*lat), prec, nrhs);
}

hisq_status hisq_pack_links(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, const void *fat_c128,
                            const void *naik_c128, void *packed, void *stream) {
    TRY(check_lattice(lat));
    TRY(check_prec(prec));
    TRY(check_ptr(fat_c128, "fat_c128"));
    TRY(check_ptr(naik_c128, "naik_c128"));
    TRY(check_ptr(packed, "packed"));
    TRY(set_device(ctx));
    int bad = 0;
    const hipError_t e = launch_pack_links(make_geom(*lat), prec, fat_c128, naik_c128, packed,
                                           static_cast<hipStream_t>(stream), &bad);
    if (e != hipSuccess)
        return device_fail(e, "pack_links");
    if (bad)
        return fail(HISQ_ERR_INVALID_ARG,
                    prec == HISQ_FP64W14 || prec == HISQ_FP32W14
                        ? "a Naik link is not of the form z conj(row 0 x row 1) in its row 2 (not a multiple "
                          "of a U(3) matrix): use an uncompressed format"
                        : "a link is not special unitary (its row 2 is not conj(row 0 x row 1)): use an "
                          "uncompressed format, or HISQ_FP64W14 / HISQ_FP32W14 for U(3) Naik links");
    return HISQ_OK;
}

hisq_status hisq_unpack_links(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, const void *packed,
                              void *fat_c128, void *naik_c128, void *stream) {
    TRY(check_lattice(lat));
    TRY(check_prec(prec));
    TRY(check_ptr(packed, "packed"));
    TRY(check_ptr(fat_c128, "fat_c128"));
    TRY(check_ptr(naik_c128, "naik_c128"));
    TRY(set_device(ctx));
    const hipError_t e = launch_unpack_links(make_geom(*lat), prec, packed, fat_c128, naik_c128,
                                             static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HISQ_OK : device_fail(e, "unpack_links");
}

hisq_status hisq_pack_field(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, int32_t nrhs,
                            const void *half_c128, void *packed, void *stream) {
    TRY(check_lattice(lat));
    TRY(check_prec(prec));
    TRY(check_nrhs(nrhs));
    TRY(check_ptr(half_c128, "half_c128"));
    TRY(check_ptr(packed, "packed"));
    TRY(set_device(ctx));
    const hipError_t e =
        launch_pack_field(make_geom(*lat), field_prec_of(prec), nrhs, half_c128, packed, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HISQ_OK : device_fail(e, "pack_field");
}

hisq_status hisq_unpack_field(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, int32_t nrhs,
                              const void *packed, void *half_c128, void *stream) {
    TRY(check_lattice(lat));
    TRY(check_prec(prec));
    TRY(check_nrhs(nrhs));
    TRY(check_ptr(packed, "packed"));
    TRY(check_ptr(half_c128, "half_c128"));
    TRY(set_device(ctx));
    const hipError_t e =
        launch_unpack_field(make_geom(*lat), field_prec_of(prec), nrhs, packed, half_c128,
                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HISQ_OK : device_fail(e, "unpack_field");
}

hisq_status hisq_dslash(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, int32_t out_parity,
                        const void *links, const void *in, void *out, int32_t nrhs, void *stream) {
    TRY(check_lattice(lat));
    TRY(check_prec(prec));
    TRY(check_nrhs(nrhs));
    if (out_parity != 0 && out_parity != 1)
        return fail(HISQ_ERR_INVALID_ARG, "out_parity = %d must be 0 or 1", out_parity);
    TRY(check_ptr(links, "links"));
    TRY(check_ptr(in, "in"));
    TRY(check_ptr(out, "out"));
    if (in == out)
        return fail(HISQ_ERR_INVALID_ARG, "in and out must not alias");
    TRY(set_device(ctx));
    DslashParams prm{};
    prm.g = make_geom(*lat);
    prm.out_parity = out_parity;
    prm.nrhs = nrhs;
    prm.links = static_cast<const char *>(links);
    prm.in = in;
    prm.out = out;
    const DslashShape s = pick_shape(ctx, prm.g, prec, field_prec_of(prec), nrhs);
    const hipError_t e = launch_dslash(prm, prec, field_prec_of(prec), EPI_PLAIN, s, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HISQ_OK : device_fail(e, "dslash");
}

hisq_status hisq_apply_m(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, double mass,
                         const void *links, const void *in_even, void *out_even, void *tmp_odd, int32_t nrhs,
                         void *stream) {
    TRY(check_lattice(lat));
    TRY(check_prec(prec));
    TRY(check_nrhs(nrhs));
    TRY(check_ptr(links, "links"));
    TRY(check_ptr(in_even, "in_even"));
    TRY(check_ptr(out_even, "out_even"));
    TRY(check_ptr(tmp_odd, "tmp_odd"));
    if (in_even == out_even || tmp_odd == in_even || tmp_odd == out_even)
        return fail(HISQ_ERR_INVALID_ARG, "in_even, out_even and tmp_odd must be distinct");
    if (!(mass == mass) || mass * mass <= 0.0)
        return fail(HISQ_ERR_INVALID_ARG, "mass^2 must be positive (mass = %g)", mass);
    TRY(set_device(ctx));
    const hipStream_t st = static_cast<hipStream_t>(stream);
    DslashParams prm{};
    prm.g = make_geom(*lat);
    prm.nrhs = nrhs;
    prm.links = static_cast<const char *>(links);
    const DslashShape s = pick_shape(ctx, prm.g, prec, field_prec_of(prec), nrhs);
    prm.out_parity = 1;
    prm.in = in_even;
    prm.out = tmp_odd;
    hipError_t e = launch_dslash(prm, prec, field_prec_of(prec), EPI_PLAIN, s, st);
    if (e != hipSuccess)
        return device_fail(e, "apply_m (D_oe)");
    prm.out_parity = 0;
    prm.in = tmp_odd;
    prm.out = out_even;
    prm.y = in_even;
    prm.ad = -1.0;
    prm.ay = mass * mass;
    e = launch_dslash(prm, prec, field_prec_of(prec), EPI_AXPY, s, st);
    return e == hipSuccess ? HISQ_OK : device_fail(e, "apply_m (D_eo)");
}

size_t hisq_apply_m_dot_workspace_bytes(const hisq_lattice *lat, int32_t nrhs) {
    if (check_lattice(lat) != HISQ_OK || check_nrhs(nrhs) != HISQ_OK)
        return 0;
    return apply_m_dot_partials_max(make_geom(*lat), nrhs) * sizeof(double);
}

hisq_status hisq_apply_m_dot(hisq_context *ctx, const hisq_lattice *lat, hisq_prec link_prec, hisq_prec field_prec,
                             double mass, const void *links, const void *in_even, void *out_even, void *tmp_odd,
                             int32_t nrhs, double *dot_out, void *ws, size_t ws_bytes, void *stream) {
    ApplyMDot a;
    TRY(check_apply_m_dot(ctx, lat, link_prec, field_prec, mass, links, in_even, out_even, tmp_odd, nrhs, dot_out,
                          &a));
    TRY(check_ptr(ws, "ws"));
    const size_t need = a.partials * sizeof(double);
    if (ws_bytes < need)
        return fail(HISQ_ERR_WORKSPACE, "workspace holds %zu bytes, needs %zu", ws_bytes, need);
    TRY(set_device(ctx));
    return run_apply_m_dot(a, static_cast<double *>(ws), static_cast<hipStream_t>(stream));
}

hisq_status hisq_stream_copy(hisq_context *ctx, const void *src, void *dst, size_t bytes, void *stream) {
    TRY(check_ptr(src, "src"));
    TRY(check_ptr(dst, "dst"));
    if (bytes == 0 || bytes % 16 != 0)
        return fail(HISQ_ERR_INVALID_ARG, "bytes = %zu must be a positive multiple of 16", bytes);
    if (reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
        return fail(HISQ_ERR_INVALID_ARG, "src and dst must be 16-byte aligned");
    const char *s0 = static_cast<const char *>(src);
    const char *d0 = static_cast<const char *>(dst);
    if (s0 < d0 + bytes && d0 < s0 + bytes)
        return fail(HISQ_ERR_INVALID_ARG, "src and dst overlap");
    TRY(set_device(ctx));
    const hipError_t e = launch_stream_copy(src, dst, bytes / 16, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HISQ_OK : device_fail(e, "stream_copy");
}

size_t hisq_stream_read_sink_words(size_t bytes) { return bytes % 16 != 0 ? 0 : stream_read_blocks(bytes / 16); }

hisq_status hisq_stream_read(hisq_context *ctx, const void *src, size_t bytes, uint32_t *sink, void *stream) {
    TRY(check_ptr(src, "src"));
    TRY(check_ptr(sink, "sink"));
    if (bytes == 0 || bytes % 16 != 0)
        return fail(HISQ_ERR_INVALID_ARG, "bytes = %zu must be a positive multiple of 16", bytes);
    if (reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(sink) % 4 != 0)
        return fail(HISQ_ERR_INVALID_ARG, "src must be 16-byte and sink 4-byte aligned");
    const char *s0 = static_cast<const char *>(src);
    const char *k0 = reinterpret_cast<const char *>(sink);
    const size_t kb = 4 * stream_read_blocks(bytes / 16);
    if (s0 < k0 + kb && k0 < s0 + bytes)
        return fail(HISQ_ERR_INVALID_ARG, "src and sink overlap");
    TRY(set_device(ctx));
    const hipError_t e = launch_stream_read(src, bytes / 16, sink, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HISQ_OK : device_fail(e, "stream_read");
}

}  // extern "C"
