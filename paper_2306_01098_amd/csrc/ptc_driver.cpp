// C ABI of the PTC preconditioner network: apply, backward, Adam, and one
// training step (forward, loss, backward over a batch of (source, solution)
// pairs, then Adam), all on the caller's device buffers.
#include <cmath>

#include "api_util.hpp"
#include "dslash.hpp"
#include "ptc.hpp"

namespace hisq {

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct PtcLayout {
    size_t a0, a1, a2, a3, g3, g2, g1, g0, partials, grad, scal, e, t, ae, src, total;
};

PtcLayout ptc_layout(const Geom &g) {
    PtcLayout L;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = a256(off + b);
        return o;
    };
    const size_t f1 = ptc_field_bytes(g, 1), f8 = ptc_field_bytes(g, PTC_CH);
    L.a0 = take(f1);
    L.a1 = take(f8);
    L.a2 = take(f8);
    L.a3 = take(f1);
    L.g3 = take(f1);
    L.g2 = take(f8);
    L.g1 = take(f8);
    L.g0 = take(f1);
    const size_t per_block = (size_t)PTC_CH * PTC_PATHS * 2 * PTC_CH;  // largest layer
    L.partials = take(sizeof(double) * per_block * ptc_blocks(g));
    L.grad = take(sizeof(double2) * PTC_NW);
    L.scal = take(sizeof(double) * 64);
    const size_t h32 = field_bytes(g, HISQ_FP32, 1);
    L.e = take(h32);
    L.t = take(h32);
    L.ae = take(h32);
    L.src = take(h32);  // the training step's current source as a one-column field
    L.total = off;
    return L;
}

struct Ptc {
    Geom g;
    PtcLayout L;
    char *ws;
    const char *links;
    hipStream_t st;
    template <typename T> T *at(size_t o) const { return reinterpret_cast<T *>(ws + o); }
};

// skip (nullable): every launch does nothing while *skip != 0.
hipError_t forward(const Ptc &P, const float2 *w, const void *in_even, void *out_even,
                   const int *skip = nullptr) {
    hipError_t e = ptc_embed(P.g, in_even, P.at<void>(P.L.a0), P.st, skip);
    if (e == hipSuccess)
        e = ptc_layer_fwd(P.g, 1, PTC_CH, P.links, w + PTC_W1, P.at<void>(P.L.a0), P.at<void>(P.L.a1), P.st,
                          skip);
    if (e == hipSuccess)
        e = ptc_layer_fwd(P.g, PTC_CH, PTC_CH, P.links, w + PTC_W2, P.at<void>(P.L.a1), P.at<void>(P.L.a2), P.st,
                          skip);
    if (e == hipSuccess)
        e = ptc_layer_fwd(P.g, PTC_CH, 1, P.links, w + PTC_W3, P.at<void>(P.L.a2), P.at<void>(P.L.a3), P.st,
                          skip);
    if (e == hipSuccess && out_even)
        e = ptc_extract(P.g, P.at<void>(P.L.a3), out_even, P.st, skip);
    return e;
}

// From the output gradient in g3 (whole lattice): weight gradients += into
// grad, input gradient (even sites) into g_in_even if non-NULL.
hipError_t backward(const Ptc &P, const float2 *w, double2 *grad, void *g_in_even) {
    double *part = P.at<double>(P.L.partials);
    hipError_t e = ptc_layer_bwd_w(P.g, PTC_CH, 1, P.links, P.at<void>(P.L.a2), P.at<void>(P.L.g3), part,
                                   grad + PTC_W3, P.st);
    if (e == hipSuccess)
        e = ptc_layer_bwd_in(P.g, PTC_CH, 1, P.links, w + PTC_W3, P.at<void>(P.L.g3), P.at<void>(P.L.g2), P.st);
    if (e == hipSuccess)
        e = ptc_layer_bwd_w(P.g, PTC_CH, PTC_CH, P.links, P.at<void>(P.L.a1), P.at<void>(P.L.g2), part,
                            grad + PTC_W2, P.st);
    if (e == hipSuccess)
        e = ptc_layer_bwd_in(P.g, PTC_CH, PTC_CH, P.links, w + PTC_W2, P.at<void>(P.L.g2), P.at<void>(P.L.g1),
                             P.st);
    if (e == hipSuccess)
        e = ptc_layer_bwd_w(P.g, 1, PTC_CH, P.links, P.at<void>(P.L.a0), P.at<void>(P.L.g1), part, grad + PTC_W1,
                            P.st);
    if (e == hipSuccess && g_in_even) {
        e = ptc_layer_bwd_in(P.g, 1, PTC_CH, P.links, w + PTC_W1, P.at<void>(P.L.g1), P.at<void>(P.L.g0), P.st);
        if (e == hipSuccess)
            e = ptc_extract(P.g, P.at<void>(P.L.g0), g_in_even, P.st);
    }
    return e;
}

hisq_status common_checks(const hisq_lattice *lat, const void *links, const void *w, const void *ws, size_t ws_bytes,
                          Ptc *P, hisq_context *ctx, void *stream) {
    hisq_status s = check_lattice(lat);
    if (s == HISQ_OK) s = check_ptr(links, "links_f32");
    if (s == HISQ_OK) s = check_ptr(w, "weights");
    if (s == HISQ_OK) s = check_ptr(ws, "ws");
    if (s == HISQ_OK) s = set_device(ctx);
    if (s != HISQ_OK)
        return s;
    P->g = make_geom(*lat);
    P->L = ptc_layout(P->g);
    if (ws_bytes < P->L.total)
        return fail(HISQ_ERR_WORKSPACE, "workspace holds %zu bytes, needs %zu", ws_bytes, P->L.total);
    P->ws = static_cast<char *>(const_cast<void *>(ws));
    P->links = static_cast<const char *>(links);
    P->st = static_cast<hipStream_t>(stream);
    return HISQ_OK;
}

}  // namespace

// Internal entry used by the flexible CG: z = N(r) on even sites; the launches
// do nothing while skip (nullable) points to a nonzero value.
hisq_status ptc_apply_internal(const hisq_lattice *lat, const void *links_f32, const void *weights, const void *in,
                               void *out, void *ws, size_t ws_bytes, hipStream_t st, const int *skip) {
    Ptc P;
    hisq_status s = common_checks(lat, links_f32, weights, ws, ws_bytes, &P, nullptr, st);
    if (s != HISQ_OK)
        return s;
    const hipError_t e = forward(P, static_cast<const float2 *>(weights), in, out, skip);
    return e == hipSuccess ? HISQ_OK : device_fail(e, "ptc forward");
}

size_t ptc_workspace(const Geom &g) { return ptc_layout(g).total; }

}  // namespace hisq

using namespace hisq;

extern "C" {

size_t hisq_ptc_workspace_bytes(const hisq_lattice *lat) {
    if (check_lattice(lat) != HISQ_OK)
        return 0;
    return ptc_layout(make_geom(*lat)).total;
}

hisq_status hisq_ptc_forward(hisq_context *ctx, const hisq_lattice *lat, const void *links_f32, const void *weights,
                             const void *in_even, void *out_even, void *ws, size_t ws_bytes, void *stream) {
    Ptc P;
    hisq_status s = common_checks(lat, links_f32, weights, ws, ws_bytes, &P, ctx, stream);
    if (s == HISQ_OK) s = check_ptr(in_even, "in_even");
    if (s == HISQ_OK) s = check_ptr(out_even, "out_even");
    if (s != HISQ_OK)
        return s;
    const hipError_t e = forward(P, static_cast<const float2 *>(weights), in_even, out_even);
    return e == hipSuccess ? HISQ_OK : device_fail(e, "ptc forward");
}

hisq_status hisq_ptc_backward(hisq_context *ctx, const hisq_lattice *lat, const void *links_f32,
                              const void *weights, const void *g_out_even, void *g_in_even, void *grad, void *ws,
                              size_t ws_bytes, void *stream) {
    Ptc P;
    hisq_status s = common_checks(lat, links_f32, weights, ws, ws_bytes, &P, ctx, stream);
    if (s == HISQ_OK) s = check_ptr(g_out_even, "g_out_even");
    if (s == HISQ_OK) s = check_ptr(grad, "grad");
    if (s != HISQ_OK)
        return s;
    // output gradient: even sites from the caller, zero on odd sites
    hipError_t e = ptc_embed(P.g, g_out_even, P.at<void>(P.L.g3), P.st);
    if (e == hipSuccess)
        e = backward(P, static_cast<const float2 *>(weights), static_cast<double2 *>(grad), g_in_even);
    return e == hipSuccess ? HISQ_OK : device_fail(e, "ptc backward");
}

hisq_status hisq_ptc_adam_step(hisq_context *ctx, void *w_master, void *w_f32, const void *grad, void *m, void *v,
                               int32_t step, double lr, double beta1, double beta2, double eps, void *stream) {
    hisq_status s = check_ptr(w_master, "w_master");
    if (s == HISQ_OK) s = check_ptr(w_f32, "w_f32");
    if (s == HISQ_OK) s = check_ptr(grad, "grad");
    if (s == HISQ_OK) s = check_ptr(m, "m");
    if (s == HISQ_OK) s = check_ptr(v, "v");
    if (s == HISQ_OK && step < 1)
        s = fail(HISQ_ERR_INVALID_ARG, "step = %d must be >= 1", step);
    if (s == HISQ_OK && !(lr > 0.0 && beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0))
        s = fail(HISQ_ERR_INVALID_ARG, "invalid Adam hyper-parameters");
    if (s == HISQ_OK) s = set_device(ctx);
    if (s != HISQ_OK)
        return s;
    const hipError_t e = ptc_adam(static_cast<double2 *>(w_master), static_cast<float2 *>(w_f32),
                                  static_cast<const double2 *>(grad), static_cast<double2 *>(m),
                                  static_cast<double2 *>(v), step, lr, beta1, beta2, eps,
                                  static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HISQ_OK : device_fail(e, "ptc adam");
}

hisq_status hisq_ptc_train_step(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f32,
                                void *w_master, void *w_f32, void *m, void *v, int32_t step, int32_t batch,
                                const void *src_f32, const void *sol_f64, double lr, double beta1, double beta2,
                                double eps, double *loss, void *ws, size_t ws_bytes, void *stream) {
    Ptc P;
    hisq_status s = common_checks(lat, links_f32, w_f32, ws, ws_bytes, &P, ctx, stream);
    if (s == HISQ_OK) s = check_ptr(src_f32, "src_f32");
    if (s == HISQ_OK) s = check_ptr(sol_f64, "sol_f64");
    if (s == HISQ_OK && batch < 1)
        s = fail(HISQ_ERR_INVALID_ARG, "batch = %d must be >= 1", batch);
    if (s == HISQ_OK && (!std::isfinite(mass) || mass * mass <= 0.0))
        s = fail(HISQ_ERR_INVALID_ARG, "mass^2 must be positive (mass = %g)", mass);
    if (s != HISQ_OK)
        return s;
    const float2 *w = static_cast<const float2 *>(w_f32);
    double2 *grad = P.at<double2>(P.L.grad);
    double *scal = P.at<double>(P.L.scal);  // [0] <x, b>, [1] loss, [2] <e, A e>
    const size_t c64 = field_bytes(P.g, HISQ_FP64, 1);
    const DslashShape shape = pick_shape(ctx, P.g, HISQ_FP32, HISQ_FP32, 1);
    hipError_t e = ptc_fill_f64(reinterpret_cast<double *>(grad), 2 * PTC_NW, P.st);
    if (e == hipSuccess) e = ptc_fill_f64(scal, 16, P.st);
    const void *src = P.at<void>(P.L.src);
    for (int k = 0; k < batch && e == hipSuccess; ++k) {
        // source k: column k of the batch-column FP32 field src_f32
        e = launch_copy_col(P.g.vh, HISQ_FP32, batch, k, src_f32, P.at<void>(P.L.src), P.st);
        const char *sol = static_cast<const char *>(sol_f64) + k * c64;
        if (e == hipSuccess)
            e = forward(P, w, src, nullptr);
        if (e == hipSuccess)
            e = ptc_xb(P.g, sol, src, P.at<double>(P.L.partials), scal + 0, P.st);
        if (e == hipSuccess)
            e = ptc_diff(P.g, P.at<void>(P.L.a3), sol, P.at<void>(P.L.e), P.st);
        // A e = m^2 e - D_eo D_oe e (FP32 links) with <e, A e>
        DslashParams prm{};
        prm.g = P.g;
        prm.nrhs = 1;
        prm.links = P.links;
        prm.out_parity = 1;
        prm.in = P.at<void>(P.L.e);
        prm.out = P.at<void>(P.L.t);
        if (e == hipSuccess) e = launch_dslash(prm, HISQ_FP32, HISQ_FP32, EPI_PLAIN, shape, P.st);
        prm.out_parity = 0;
        prm.in = P.at<void>(P.L.t);
        prm.out = P.at<void>(P.L.ae);
        prm.y = P.at<void>(P.L.e);
        prm.ad = -1.0;
        prm.ay = mass * mass;
        prm.partials = P.at<double>(P.L.partials);
        prm.dot_out = scal + 2;
        prm.dot_stride = 1;
        if (e == hipSuccess) e = launch_dslash(prm, HISQ_FP32, HISQ_FP32, EPI_AXPY_DOT, shape, P.st);
        if (e == hipSuccess)
            e = ptc_energy_grad(P.g, P.at<void>(P.L.ae), scal + 2, scal + 0, 1.0 / batch, P.at<void>(P.L.g3),
                                scal + 1, P.st);
        if (e == hipSuccess)
            e = backward(P, w, grad, nullptr);
    }
    if (e == hipSuccess)
        e = ptc_adam(static_cast<double2 *>(w_master), static_cast<float2 *>(w_f32), grad,
                     static_cast<double2 *>(m), static_cast<double2 *>(v), step, lr, beta1, beta2, eps, P.st);
    if (e == hipSuccess && loss) {
        e = hipMemcpyAsync(loss, scal + 1, sizeof(double), hipMemcpyDeviceToHost, P.st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(P.st);
    }
    return e == hipSuccess ? HISQ_OK : device_fail(e, "ptc train step");
}

}  // extern "C"
