// Vector kernels of flexible CG with a (possibly non-symmetric) preconditioner:
// complex inner products, and updates with complex alpha, beta.
#include "fcg.hpp"
#include "internal.hpp"
#include "reduce.hpp"

namespace hisq {

namespace {

constexpr int FB = 256;

// Block partials of <a, b> = sum conj(a) b of two FP32 even fields (FP64
// sums): real parts in partials[0 .. nblk), imaginary in [nblk .. 2 nblk).
__global__ void __launch_bounds__(FB) dot_kernel(int vh, const void *a, const void *b, double *partials,
                                                 const int *skip) {
    if (skip && *skip)
        return;
    __shared__ double lds[8];
    const int i = blockIdx.x * FB + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (i < vh) {
        cplx<float> x[3], y[3];
        FieldIO<HISQ_FP32>::template load<float>(a, vh, 1, 0, i, x);
        FieldIO<HISQ_FP32>::template load<float>(b, vh, 1, 0, i, y);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[0] += (double)x[c].re * y[c].re + (double)x[c].im * y[c].im;
            v[1] += (double)x[c].re * y[c].im - (double)x[c].im * y[c].re;
        }
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = v[0];
        partials[gridDim.x + blockIdx.x] = v[1];
    }
}

// alpha = <p, r> / <p, A p>; x += alpha p (FP64), r -= alpha q, and block
// partials of ||r||^2.
__global__ void __launch_bounds__(FB) xr_kernel(int vh, void *x, const void *p, const void *q, void *r,
                                                const FcgScalars *s, double *partials) {
    __shared__ double lds[4];
    const FcgScalars st = *s;
    const bool ok = st.active && st.pq > 0.0 && st.pq < 1e308;
    const double ar = ok ? st.pr.x / st.pq : 0.0, ai = ok ? st.pr.y / st.pq : 0.0;
    const int i = blockIdx.x * FB + threadIdx.x;
    double part[1] = {0.0};
    if (ok && i < vh) {
        cplx<float> pv[3], qv[3], rv[3];
        cplx<double> xv[3];
        FieldIO<HISQ_FP32>::template load<float>(p, vh, 1, 0, i, pv);
        FieldIO<HISQ_FP32>::template load<float>(q, vh, 1, 0, i, qv);
        FieldIO<HISQ_FP32>::template load<float>(r, vh, 1, 0, i, rv);
        FieldIO<HISQ_FP64>::template load<double>(x, vh, 1, 0, i, xv);
        const float fr = (float)ar, fi = (float)ai;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cmac(xv[c], ar, ai, cplx<double>{(double)pv[c].re, (double)pv[c].im});
            cmac(rv[c], -fr, -fi, qv[c]);
            part[0] += (double)rv[c].re * rv[c].re + (double)rv[c].im * rv[c].im;
        }
        FieldIO<HISQ_FP64>::template store<double>(x, vh, 1, 0, i, xv);
        FieldIO<HISQ_FP32>::template store<float>(r, vh, 1, 0, i, rv);
    }
    block_sum<1>(part, lds);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = part[0];
}

// One block: sums the ||r||^2 partials of xr_kernel, advances the scalars
// and raises the flags; sets the launch flags skip (not active) and nopend (no
// true residual pending).
__global__ void __launch_bounds__(FB) xr_finalize_kernel(FcgScalars *s, const double *partials, int nblk,
                                                         int *flags) {
    __shared__ double tot;
    sum_partials_block(partials, 1, nblk, &tot);
    if (threadIdx.x != 0)
        return;
    FcgScalars n = *s;
    if (!n.active)
        return;
    const bool ok = n.pq > 0.0 && n.pq < 1e308;
    if (!ok) {
        n.flag = FLAG_BREAKDOWN;
        n.active = 0;
    } else {
        n.iters += 1;
        n.rho = tot;
        if (!(tot == tot)) {
            n.flag = FLAG_BREAKDOWN;
            n.active = 0;
        } else if (tot <= n.target2) {
            n.flag = FLAG_CONV;
            n.active = 0;
        } else if (n.delta2 > 0.0 && tot < n.delta2 * n.rmax2) {
            n.flag = FLAG_RELIABLE;
            n.active = 0;
        } else if (n.iters >= n.max_iter) {
            n.flag = FLAG_MAXIT;
            n.active = 0;
        } else {
            n.rmax2 = fmax(n.rmax2, tot);
        }
    }
    *s = n;
    flags[FCG_SKIP] = n.active ? 0 : 1;
    flags[FCG_NOPEND] = (n.flag == FLAG_CONV || n.flag == FLAG_RELIABLE) && !n.active ? 0 : 1;
}

// The decision after the FP64 true residual of a waiting solve (its block
// partials in trpart): done, iteration limit, breakdown, or residual
// replacement (the recurrence goes on from the replaced r: the direction is
// rebuilt from z = N(r) by the launches that follow, gated by norestart).
// Every check block runs it: with nothing pending it only clears norestart.
__global__ void __launch_bounds__(FB) fcg_restart_kernel(FcgScalars *s, const double *trpart, int nblk,
                                                         int *flags) {
    __shared__ double tot;
    const bool pend = flags[FCG_NOPEND] == 0;
    if (pend)
        sum_partials_block(trpart, 1, nblk, &tot);
    if (threadIdx.x != 0)
        return;
    if (!pend) {
        flags[FCG_NORESTART] = 1;
        return;
    }
    FcgScalars n = *s;
    const double r2 = tot;
    n.rtrue2 = r2;
    int replaced = 0;
    if (!(r2 >= 0.0 && r2 < 1.0e308)) {
        n.flag = FLAG_BREAKDOWN;
    } else if (r2 <= n.target2) {
        n.flag = FLAG_DONE;
    } else if (n.iters >= n.max_iter) {
        n.flag = FLAG_MAXIT;
    } else {
        n.nrel += 1;
        n.rho = r2;
        n.rmax2 = r2;
        n.flag = FLAG_RUN;
        n.active = 1;
        replaced = 1;
    }
    *s = n;
    flags[FCG_SKIP] = n.active ? 0 : 1;
    flags[FCG_NOPEND] = 1;
    flags[FCG_NORESTART] = replaced ? 0 : 1;
}

// beta = <A p, z> / <p, A p>;  p = z - beta p.
__global__ void __launch_bounds__(FB) p_kernel(int vh, const void *z, void *p, const FcgScalars *s,
                                               const int *skip) {
    if (skip && *skip)
        return;
    const FcgScalars st = *s;
    const int i = blockIdx.x * FB + threadIdx.x;
    if (!st.active || i >= vh)
        return;
    const float br = (float)(st.qz.x / st.pq), bi = (float)(st.qz.y / st.pq);
    cplx<float> zv[3], pv[3];
    FieldIO<HISQ_FP32>::template load<float>(z, vh, 1, 0, i, zv);
    FieldIO<HISQ_FP32>::template load<float>(p, vh, 1, 0, i, pv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<float> o = zv[c];
        cmac(o, -br, -bi, pv[c]);
        pv[c] = o;
    }
    FieldIO<HISQ_FP32>::template store<float>(p, vh, 1, 0, i, pv);
}

}  // namespace

hipError_t launch_fcg_dot(int vh, const void *a, const void *b, double *partials, double2 *out, hipStream_t st,
                          const int *skip) {
    const int nblk = (vh + FB - 1) / FB;
    dot_kernel<<<nblk, FB, 0, st>>>(vh, a, b, partials, skip);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? launch_sum_partials(partials, 2, nblk, reinterpret_cast<double *>(out), 1, skip, st)
                           : e;
}

hipError_t launch_fcg_xr(int vh, void *x, const void *p, const void *q, void *r, FcgScalars *s, double *partials,
                         int *flags, hipStream_t st) {
    const int nblk = (vh + FB - 1) / FB;
    xr_kernel<<<nblk, FB, 0, st>>>(vh, x, p, q, r, s, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    xr_finalize_kernel<<<1, FB, 0, st>>>(s, partials, nblk, flags);
    return hipGetLastError();
}

hipError_t launch_fcg_restart(int vh, FcgScalars *s, const double *trpart, int *flags, hipStream_t st) {
    fcg_restart_kernel<<<1, FB, 0, st>>>(s, trpart, (vh + FB - 1) / FB, flags);
    return hipGetLastError();
}

hipError_t launch_fcg_p(int vh, const void *z, void *p, const FcgScalars *s, hipStream_t st, const int *skip) {
    p_kernel<<<(vh + FB - 1) / FB, FB, 0, st>>>(vh, z, p, s, skip);
    return hipGetLastError();
}

}  // namespace hisq
