// Host driver of flexible CG (Notay's FCG with one-vector truncation) with
// the PTC network as preconditioner: FP32 iteration vectors and links, FP64
// solution, FP64 inner products and FP64 reliable updates (residual
// replacement by the FP64 true residual, the recurrence continuing from it).
#include <chrono>
#include <cmath>
#include <vector>

#include "api_util.hpp"
#include "dslash.hpp"
#include "fcg.hpp"

namespace hisq {

size_t ptc_workspace(const Geom &g);
hisq_status ptc_apply_internal(const hisq_lattice *lat, const void *links_f32, const void *weights, const void *in,
                               void *out, void *ws, size_t ws_bytes, hipStream_t st);

namespace {

size_t f256(size_t x) { return (x + 255) & ~(size_t)255; }

struct FcgLayout {
    size_t state, flags, scal, partials, r, p, q, t, z, ax, t64, ptc, total;
};

FcgLayout fcg_layout(const Geom &g) {
    FcgLayout L;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = f256(off + b);
        return o;
    };
    L.state = take(sizeof(FcgScalars));
    L.flags = take(64 * sizeof(unsigned));
    L.scal = take(64 * sizeof(double));
    L.partials = take(sizeof(double) * 2 * (size_t)(g.vh / 16 + 64));
    const size_t f32 = field_bytes(g, HISQ_FP32, 1), f64 = field_bytes(g, HISQ_FP64, 1);
    L.r = take(f32);
    L.p = take(f32);
    L.q = take(f32);
    L.t = take(f32);
    L.z = take(f32);
    L.ax = take(f64);
    L.t64 = take(f64);
    L.ptc = take(ptc_workspace(g));
    L.total = off;
    return L;
}

double fnow() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); }

}  // namespace

}  // namespace hisq

using namespace hisq;

extern "C" {

size_t hisq_fcg_workspace_bytes(const hisq_lattice *lat) {
    if (check_lattice(lat) != HISQ_OK)
        return 0;
    return fcg_layout(make_geom(*lat)).total;
}

hisq_status hisq_fcg(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                     const void *links_f32, const void *weights, const void *b, void *x, double tol,
                     int32_t max_iter, void *ws, size_t ws_bytes, hisq_solve_info *info, void *stream) {
    const double t0 = fnow();
    hisq_status s = check_lattice(lat);
    if (s == HISQ_OK) s = check_ptr(links_f64, "links_f64");
    if (s == HISQ_OK) s = check_ptr(links_f32, "links_f32");
    if (s == HISQ_OK) s = check_ptr(weights, "weights");
    if (s == HISQ_OK) s = check_ptr(b, "b");
    if (s == HISQ_OK) s = check_ptr(x, "x");
    if (s == HISQ_OK) s = check_ptr(ws, "ws");
    if (s == HISQ_OK && (!std::isfinite(mass) || mass * mass <= 0.0))
        s = fail(HISQ_ERR_INVALID_ARG, "mass^2 must be positive (mass = %g)", mass);
    if (s == HISQ_OK && !(tol > 0.0 && tol < 1.0))
        s = fail(HISQ_ERR_INVALID_ARG, "tol = %g must be in (0, 1)", tol);
    if (s == HISQ_OK && max_iter < 1)
        s = fail(HISQ_ERR_INVALID_ARG, "max_iter = %d must be >= 1", max_iter);
    if (s == HISQ_OK && b == x)
        s = fail(HISQ_ERR_INVALID_ARG, "b and x must not alias");
    if (s == HISQ_OK) s = set_device(ctx);
    if (s != HISQ_OK)
        return s;
    const Geom g = make_geom(*lat);
    const FcgLayout L = fcg_layout(g);
    if (ws_bytes < L.total)
        return fail(HISQ_ERR_WORKSPACE, "workspace holds %zu bytes, needs %zu", ws_bytes, L.total);
    char *W = static_cast<char *>(ws);
    hipStream_t st = static_cast<hipStream_t>(stream);
    FcgScalars *ds = reinterpret_cast<FcgScalars *>(W + L.state);
    unsigned *flags = reinterpret_cast<unsigned *>(W + L.flags);
    double *scal = reinterpret_cast<double *>(W + L.scal);
    double *partials = reinterpret_cast<double *>(W + L.partials);
    void *r = W + L.r, *p = W + L.p, *q = W + L.q, *t = W + L.t, *z = W + L.z, *ax = W + L.ax, *t64 = W + L.t64;
    const DslashShape sh64 = pick_shape(ctx, g, HISQ_FP64, HISQ_FP64, 1);
    const DslashShape sh32 = pick_shape(ctx, g, HISQ_FP32, HISQ_FP32, 1);
    const double m2 = mass * mass;
    auto dev = [](hipError_t e, const char *w) { return e == hipSuccess ? HISQ_OK : device_fail(e, w); };

    // rtrue2 = ||b - M x||^2, r = b - M x (FP32 copy)
    auto true_residual = [&](double *rtrue2) -> hisq_status {
        DslashParams prm{};
        prm.g = g;
        prm.nrhs = 1;
        prm.links = static_cast<const char *>(links_f64);
        prm.out_parity = 1;
        prm.in = x;
        prm.out = t64;
        hipError_t e = launch_dslash(prm, HISQ_FP64, HISQ_FP64, EPI_PLAIN, sh64, st);
        if (e == hipSuccess) {
            prm.out_parity = 0;
            prm.in = t64;
            prm.out = ax;
            prm.y = x;
            prm.ad = -1.0;
            prm.ay = m2;
            e = launch_dslash(prm, HISQ_FP64, HISQ_FP64, EPI_AXPY, sh64, st);
        }
        if (e == hipSuccess)
            e = launch_residual(g.vh, HISQ_FP32, b, ax, r, partials, scal + 0, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rtrue2, scal + 0, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        return dev(e, "fcg true residual");
    };
    auto precondition = [&]() -> hisq_status {  // z = N(r)
        return ptc_apply_internal(lat, links_f32, weights, r, z, W + L.ptc, L.total - L.ptc, st);
    };

    hipError_t e = launch_fill_u32(flags, 64, 0u, st);
    double bnorm2 = 0.0, rtrue2 = 0.0;
    if (e == hipSuccess)
        e = launch_norm2(g.vh, b, partials, scal + 1, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&bnorm2, scal + 1, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess)
        return device_fail(e, "fcg setup");
    if ((s = true_residual(&rtrue2)) != HISQ_OK)
        return s;
    FcgScalars hs{};
    hs.rho = rtrue2;
    hs.rmax2 = rtrue2;
    hs.target2 = tol * tol * bnorm2;
    hs.delta2 = 0.01;  // replace r by the true residual when it fell by 10x
    hs.max_iter = max_iter;
    int reliable = 0;
    bool done = !(rtrue2 > hs.target2);
    bool broke = !std::isfinite(rtrue2) || !std::isfinite(bnorm2);
    if (!done && !broke) {
        hs.active = 1;
        hs.flag = FLAG_RUN;
        if ((s = precondition()) != HISQ_OK)
            return s;
        e = launch_copy(g.vh, 1, HISQ_FP32, HISQ_FP32, z, p, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ds, &hs, sizeof hs, hipMemcpyHostToDevice, st);
        if (e != hipSuccess)
            return device_fail(e, "fcg start");
    }
    DslashParams prm{};
    prm.g = g;
    prm.nrhs = 1;
    prm.links = static_cast<const char *>(links_f32);
    while (!done && !broke) {
        // q = M p with Re <p, q>
        prm.out_parity = 1;
        prm.in = p;
        prm.out = t;
        prm.y = nullptr;
        prm.partials = nullptr;
        e = launch_dslash(prm, HISQ_FP32, HISQ_FP32, EPI_PLAIN, sh32, st);
        DslashParams pd = prm;
        pd.out_parity = 0;
        pd.in = t;
        pd.out = q;
        pd.y = p;
        pd.ad = -1.0;
        pd.ay = m2;
        pd.partials = partials;
        pd.dot_out = &ds->pq;
        pd.dot_stride = 1;
        if (e == hipSuccess) e = launch_dslash(pd, HISQ_FP32, HISQ_FP32, EPI_AXPY_DOT, sh32, st);
        if (e == hipSuccess) e = launch_fcg_dot(g.vh, p, r, partials, &ds->pr, st);
        if (e == hipSuccess) e = launch_fcg_xr(g.vh, x, p, q, r, ds, partials, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&hs, ds, sizeof hs, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return device_fail(e, "fcg iteration");
        if (!hs.active) {
            if (hs.flag == FLAG_BREAKDOWN) {
                broke = true;
                break;
            }
            if (hs.flag == FLAG_MAXIT)
                break;
            // CONV or RELIABLE: FP64 true residual, then finish or go on
            if ((s = true_residual(&rtrue2)) != HISQ_OK)
                return s;
            if (!std::isfinite(rtrue2)) {
                broke = true;
                break;
            }
            if (rtrue2 <= hs.target2) {
                done = true;
                break;
            }
            if (hs.iters >= max_iter)
                break;
            // residual replacement: r now holds the FP64 b - A x; the
            // recurrence goes on from it (q and <p, A p> of this iteration
            // are kept), as in reliable-update CG
            ++reliable;
            hs.rho = rtrue2;
            hs.rmax2 = rtrue2;
            hs.active = 1;
            hs.flag = FLAG_RUN;
            e = hipMemcpyAsync(ds, &hs, sizeof hs, hipMemcpyHostToDevice, st);
            if (e != hipSuccess)
                return device_fail(e, "fcg replacement");
        }
        // z = N(r); p = z - (<q, z> / <p, q>) p
        if ((s = precondition()) != HISQ_OK)
            return s;
        e = launch_fcg_dot(g.vh, q, z, partials, &ds->qz, st);
        if (e == hipSuccess) e = launch_fcg_p(g.vh, z, p, ds, st);
        if (e != hipSuccess)
            return device_fail(e, "fcg direction");
    }
    if (!done && !broke) {
        if ((s = true_residual(&rtrue2)) != HISQ_OK)
            return s;
        done = std::isfinite(rtrue2) && rtrue2 <= hs.target2;
    }
    if (info) {
        info->iterations = hs.iters;
        info->reliable_updates = reliable;
        info->true_residual = bnorm2 > 0 ? std::sqrt(rtrue2 / bnorm2) : std::sqrt(rtrue2);
        info->seconds = fnow() - t0;
        info->shared_iterations = 0;
        info->refine_iterations = 0;
    }
    if (broke)
        return fail(HISQ_ERR_BREAKDOWN, "flexible CG breakdown");
    if (!done)
        return fail(HISQ_ERR_NOT_CONVERGED, "flexible CG did not reach tol in %d iterations", max_iter);
    return HISQ_OK;
}

}  // extern "C"
