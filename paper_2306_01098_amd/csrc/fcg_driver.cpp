// Host driver of flexible CG (Notay's FCG with one-vector truncation) with
// the PTC network as preconditioner: FP32 iteration vectors and links, FP64
// solution, FP64 inner products and FP64 reliable updates (residual
// replacement by the FP64 true residual, the recurrence continuing from it).
// The device takes every decision: each iteration is followed by a check
// block whose launches are gated by flags in device memory, and chunks of
// iterations are replayed from a HIP graph; the host reads the state once per
// chunk.
#include <chrono>
#include <cmath>
#include <vector>

#include "api_util.hpp"
#include "dslash.hpp"
#include "fcg.hpp"

namespace hisq {

size_t ptc_workspace(const Geom &g);
hisq_status ptc_apply_internal(const hisq_lattice *lat, const void *links_f32, const void *weights, const void *in,
                               void *out, void *ws, size_t ws_bytes, hipStream_t st, const int *skip);

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
    L.partials = take(sizeof(double) * 2 * (size_t)(g.vh / 4 + 64));  // a Dslash site block holds >= 4 sites
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

// A private non-blocking stream ordered after the caller's stream; waited
// for and destroyed on exit.
struct FcgStream {
    hipStream_t own = nullptr;
    hipEvent_t ev = nullptr;
    hipError_t init(hipStream_t caller) {
        hipError_t e = hipStreamCreateWithFlags(&own, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventRecord(ev, caller);
        return e == hipSuccess ? hipStreamWaitEvent(own, ev, 0) : e;
    }
    ~FcgStream() {
        if (own) {
            (void)hipStreamSynchronize(own);
            (void)hipStreamDestroy(own);
        }
        if (ev)
            (void)hipEventDestroy(ev);
    }
};

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
    // a private stream ordered after the caller's (graphs cannot be captured
    // on the legacy default stream)
    FcgStream fs;
    if (hipError_t e = fs.init(static_cast<hipStream_t>(stream)); e != hipSuccess)
        return device_fail(e, "fcg stream");
    hipStream_t st = fs.own;
    FcgScalars *ds = reinterpret_cast<FcgScalars *>(W + L.state);
    int *flags = reinterpret_cast<int *>(W + L.flags);
    double *scal = reinterpret_cast<double *>(W + L.scal);
    double *partials = reinterpret_cast<double *>(W + L.partials);
    void *r = W + L.r, *p = W + L.p, *q = W + L.q, *t = W + L.t, *z = W + L.z, *ax = W + L.ax, *t64 = W + L.t64;
    const DslashShape sh64 = pick_shape(ctx, g, HISQ_FP64, HISQ_FP64, 1);
    const DslashShape sh32 = pick_shape(ctx, g, HISQ_FP32, HISQ_FP32, 1);
    const double m2 = mass * mass;
    const int *f_skip = flags + FCG_SKIP, *f_nopend = flags + FCG_NOPEND, *f_norestart = flags + FCG_NORESTART;
    auto dev = [](hipError_t e, const char *w) { return e == hipSuccess ? HISQ_OK : device_fail(e, w); };

    // r = b - M x in FP64 (FP32 copy in r) and the block partials of its
    // norm; the launches do nothing while *gate != 0 (gate nullable)
    auto residual_launches = [&](const int *gate) -> hipError_t {
        DslashParams prm{};
        prm.g = g;
        prm.nrhs = 1;
        prm.links = static_cast<const char *>(links_f64);
        prm.skip = gate;
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
        return e == hipSuccess ? launch_residual_parts(g.vh, HISQ_FP32, b, ax, r, partials, gate, st) : e;
    };
    auto precondition = [&](const int *gate) -> hisq_status {  // z = N(r)
        return ptc_apply_internal(lat, links_f32, weights, r, z, W + L.ptc, L.total - L.ptc, st, gate);
    };

    // set-up on the host: ||b||, the FP64 true residual, z = N(r), p = z
    double bnorm2 = 0.0, rtrue2 = 0.0;
    hipError_t e = launch_norm2(g.vh, b, partials, scal + 1, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&bnorm2, scal + 1, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = residual_launches(nullptr);
    if (e == hipSuccess)
        e = launch_sum_partials(partials, 1, (g.vh + 255) / 256, scal + 0, 1, nullptr, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&rtrue2, scal + 0, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return device_fail(e, "fcg setup");
    FcgScalars hs{};
    hs.rho = rtrue2;
    hs.rmax2 = rtrue2;
    hs.rtrue2 = rtrue2;
    hs.target2 = tol * tol * bnorm2;
    hs.delta2 = 0.01;  // replace r by the true residual when it fell by 10x
    hs.max_iter = max_iter;
    hs.flag = FLAG_DONE;
    bool broke = !std::isfinite(rtrue2) || !std::isfinite(bnorm2);
    if (broke)
        hs.flag = FLAG_BREAKDOWN;
    const bool start = !broke && rtrue2 > hs.target2;
    if (start) {
        hs.active = 1;
        hs.flag = FLAG_RUN;
        if ((s = precondition(nullptr)) != HISQ_OK)
            return s;
        e = launch_copy(g.vh, 1, HISQ_FP32, HISQ_FP32, z, p, st);
        const int fl[3] = {0, 1, 1};  // skip, nopend, norestart
        if (e == hipSuccess)
            e = hipMemcpyAsync(ds, &hs, sizeof hs, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(flags, fl, sizeof fl, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return device_fail(e, "fcg start");
    }

    // One iteration, then a check block, all gated on the device:
    //   q = M p with Re <p, q>; <p, r>; x += alpha p, r -= alpha q, flags;
    //   z = N(r); <q, z>; p = z - beta p                   (while running)
    //   r = b - M x in FP64 and the decision               (when flagged)
    //   z = N(r); <q, z>; p = z - beta p                   (after a replacement)
    auto step = [&]() -> hisq_status {
        DslashParams prm{};
        prm.g = g;
        prm.nrhs = 1;
        prm.links = static_cast<const char *>(links_f32);
        prm.skip = f_skip;
        prm.out_parity = 1;
        prm.in = p;
        prm.out = t;
        hipError_t e2 = launch_dslash(prm, HISQ_FP32, HISQ_FP32, EPI_PLAIN, sh32, st);
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
        if (e2 == hipSuccess) e2 = launch_dslash(pd, HISQ_FP32, HISQ_FP32, EPI_AXPY_DOT, sh32, st);
        if (e2 == hipSuccess) e2 = launch_fcg_dot(g.vh, p, r, partials, &ds->pr, st, f_skip);
        if (e2 == hipSuccess) e2 = launch_fcg_xr(g.vh, x, p, q, r, ds, partials, flags, st);
        if (e2 != hipSuccess)
            return dev(e2, "fcg iteration");
        hisq_status s2 = precondition(f_skip);
        if (s2 != HISQ_OK)
            return s2;
        e2 = launch_fcg_dot(g.vh, q, z, partials, &ds->qz, st, f_skip);
        if (e2 == hipSuccess) e2 = launch_fcg_p(g.vh, z, p, ds, st, f_skip);
        if (e2 == hipSuccess) e2 = residual_launches(f_nopend);
        if (e2 == hipSuccess) e2 = launch_fcg_restart(g.vh, ds, partials, flags, st);
        if (e2 != hipSuccess)
            return dev(e2, "fcg check");
        if ((s2 = precondition(f_norestart)) != HISQ_OK)
            return s2;
        e2 = launch_fcg_dot(g.vh, q, z, partials, &ds->qz, st, f_norestart);
        if (e2 == hipSuccess) e2 = launch_fcg_p(g.vh, z, p, ds, st, f_norestart);
        return dev(e2, "fcg direction");
    };

    // chunks of iterations captured once in a graph and replayed; the host
    // reads the state after each chunk
    const int chunk = 8;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    struct GraphGuard {
        hipGraph_t *g;
        hipGraphExec_t *x;
        ~GraphGuard() {
            if (*x) (void)hipGraphExecDestroy(*x);
            if (*g) (void)hipGraphDestroy(*g);
        }
    } gg{&graph, &exec};
    if (start) {
        e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hisq_status ls = HISQ_OK;
            for (int k = 0; k < chunk && ls == HISQ_OK; ++k)
                ls = step();
            e = hipStreamEndCapture(st, &graph);
            if (ls == HISQ_OK && e == hipSuccess)
                e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (ls != HISQ_OK || e != hipSuccess)
                exec = nullptr;
        }
        (void)hipGetLastError();
    }
    const long max_chunks = (long)max_iter / chunk + 4;
    for (long c = 0; start && c < max_chunks; ++c) {
        if (exec) {
            e = hipGraphLaunch(exec, st);
            if (e != hipSuccess)
                return device_fail(e, "fcg chunk");
        } else {
            for (int k = 0; k < chunk; ++k)
                if ((s = step()) != HISQ_OK)
                    return s;
        }
        e = hipMemcpyAsync(&hs, ds, sizeof hs, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return device_fail(e, "fcg state");
        if (!hs.active && (hs.flag == FLAG_DONE || hs.flag == FLAG_MAXIT || hs.flag == FLAG_BREAKDOWN))
            break;
    }
    broke = broke || hs.flag == FLAG_BREAKDOWN;
    bool done = hs.flag == FLAG_DONE;
    if (hs.flag == FLAG_DONE || hs.flag == FLAG_BREAKDOWN) {
        rtrue2 = hs.rtrue2;
    } else {  // stopped on the iteration limit: the true residual of the last iterate
        e = residual_launches(nullptr);
        if (e == hipSuccess)
            e = launch_sum_partials(partials, 1, (g.vh + 255) / 256, scal + 0, 1, nullptr, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&rtrue2, scal + 0, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return device_fail(e, "fcg final residual");
        done = std::isfinite(rtrue2) && rtrue2 <= hs.target2;
    }
    if (info) {
        info->iterations = hs.iters;
        info->reliable_updates = hs.nrel;
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
