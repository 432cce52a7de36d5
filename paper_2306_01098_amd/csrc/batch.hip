// Batched CG over many independent problems on lattices of different sizes.
//
// One launch covers the sites of every problem: a work list maps each block
// to (problem, first site), so 64 small solves advance together with four
// launches per iteration instead of 256, and the sequence is captured once in
// a HIP graph.  Per-problem Krylov scalars live on the device; each reducing
// kernel stores block partials and a finalize kernel (one wavefront per
// problem) sums them in a fixed order and advances the scalars.
#include "batch.hpp"
#include "dslash.hpp"
#include "reduce.hpp"

namespace hisq {

namespace {

enum { FIN_PQ = 0, FIN_XR, FIN_RESID, FIN_BNORM, FIN_RESTART };
constexpr int FIN_BLOCK = 256;  // four problems per finalize block

template <int FP> struct SloppyT;
template <> struct SloppyT<HISQ_FP64> { using T = double; };
template <> struct SloppyT<HISQ_FP32> { using T = float; };

__device__ __forceinline__ bool pos_finite(double v) { return v > 0.0 && v < 1.0e308; }

// Whether problem j takes part in a launch of the given role.
__device__ __forceinline__ bool participates(const BatchArgs &a, int j, int role) {
    return role <= ROLE_ITER_DEO ? a.st[j].active != 0 : a.mask[j] != 0;
}

// Dslash over all participating problems.
//  ROLE_ITER_DOE: t = D_oe p             (sloppy links/fields)
//  ROLE_ITER_DEO: q = m^2 p - D_eo t, Re<p, q> -> st[j].pq
//  ROLE_TRUE_DOE: t64 = D_oe x           (FP64)
//  ROLE_TRUE_DEO: ax = m^2 x - D_eo t64  (FP64)
template <int LP, int FP, int ROLE, int TB>
__global__ void __launch_bounds__(TB) batch_dslash_kernel(BatchArgs a) {
    using A = typename Prec<LP>::acc;
    if (ROLE <= ROLE_ITER_DEO && *a.nactive == 0)  // iterations stop once no problem is active
        return;
    if (ROLE > ROLE_ITER_DEO && *a.npend == 0)  // no problem waits for a true residual
        return;
    constexpr bool DOT = ROLE == ROLE_ITER_DEO;
    constexpr bool AXPY = ROLE == ROLE_ITER_DEO || ROLE == ROLE_TRUE_DEO;
    constexpr int parity = (ROLE == ROLE_ITER_DOE || ROLE == ROLE_TRUE_DOE) ? 1 : 0;
    const int blk = blockIdx.x;
    const int j = a.blk_prob[blk];
    const BatchProb &P = a.probs[j];
    const int i = (blk - P.first_blk) * TB + threadIdx.x;
    const bool go = participates(a, j, ROLE) && i < P.g.vh;
    double dot[1] = {0.0};
    if (go) {
        const char *links = ROLE <= ROLE_ITER_DEO ? P.links_in : P.links64;
        const void *in = ROLE == ROLE_ITER_DOE ? P.p : ROLE == ROLE_ITER_DEO ? P.t : ROLE == ROLE_TRUE_DOE ? P.x : P.t64;
        void *out = ROLE == ROLE_ITER_DOE ? P.t : ROLE == ROLE_ITER_DEO ? P.q : ROLE == ROLE_TRUE_DOE ? P.t64 : P.ax;
        cplx<A> acc[1][3];
        dslash_site<LP, FP, 1, A, true>(P.g, parity, links, in, i, 1, 0, 1, acc);
        if (AXPY) {
            const void *y = ROLE == ROLE_ITER_DEO ? P.p : P.x;
            cplx<A> yv[3];
            FieldIO<FP>::template load<A>(y, P.g.vh, 1, 0, i, yv);
            const A m2 = (A)P.m2;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc[0][c].re = fma(m2, yv[c].re, -acc[0][c].re);
                acc[0][c].im = fma(m2, yv[c].im, -acc[0][c].im);
                if (DOT) {
                    dot[0] = fma((double)yv[c].re, (double)acc[0][c].re, dot[0]);
                    dot[0] = fma((double)yv[c].im, (double)acc[0][c].im, dot[0]);
                }
            }
        }
        FieldIO<FP>::template store<A>(out, P.g.vh, 1, 0, i, acc[0]);
    }
    if (!DOT)
        return;
    __shared__ double lds[TB / 64];
    block_sum<1>(dot, lds);
    if (threadIdx.x == 0)
        a.partials[blk] = dot[0];
}

// x += alpha p, r -= alpha q, and block partials of <r, r>.
template <int FP, int TB>
__global__ void __launch_bounds__(TB) batch_xr_kernel(BatchArgs a) {
    using T = typename SloppyT<FP>::T;
    if (*a.nactive == 0)
        return;
    const int blk = blockIdx.x;
    const int j = a.blk_prob[blk];
    const BatchProb &P = a.probs[j];
    const int i = (blk - P.first_blk) * TB + threadIdx.x;
    const CgScalars st = a.st[j];
    const bool go = st.active && pos_finite(st.pq) && i < P.g.vh;
    double part[1] = {0.0};
    if (go) {
        const double alpha = st.rho / st.pq;
        const T al = (T)alpha;
        cplx<T> p[3], q[3], r[3];
        cplx<double> x[3];
        FieldIO<FP>::template load<T>(P.p, P.g.vh, 1, 0, i, p);
        FieldIO<FP>::template load<T>(P.q, P.g.vh, 1, 0, i, q);
        FieldIO<FP>::template load<T>(P.r, P.g.vh, 1, 0, i, r);
        FieldIO<HISQ_FP64>::template load<double>(P.x, P.g.vh, 1, 0, i, x);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[c].re = fma(alpha, (double)p[c].re, x[c].re);
            x[c].im = fma(alpha, (double)p[c].im, x[c].im);
            r[c].re = fma(-al, q[c].re, r[c].re);
            r[c].im = fma(-al, q[c].im, r[c].im);
            part[0] = fma((double)r[c].re, (double)r[c].re, part[0]);
            part[0] = fma((double)r[c].im, (double)r[c].im, part[0]);
        }
        FieldIO<HISQ_FP64>::template store<double>(P.x, P.g.vh, 1, 0, i, x);
        FieldIO<FP>::template store<T>(P.r, P.g.vh, 1, 0, i, r);
    }
    __shared__ double lds[TB / 64];
    block_sum<1>(part, lds);
    if (threadIdx.x == 0)
        a.partials[blk] = part[0];
}

// Finalize of the reducing batch kernels: one wavefront per problem sums the
// problem's block partials (deterministic, see wave_sum_slot), then its lane 0
//  FIN_PQ:    st[j].pq = total (active problems)
//  FIN_XR:    advances the problem's scalars and raises its flags; a problem
//             that stops leaves the active count (and is stamped with the
//             device clock, restamped below when its true residual confirms it)
//  FIN_RESID: st[j].rho_new = total (masked problems)
//  FIN_BNORM: bnorm2[j] = total
//  FIN_RESTART (no partials): the true-residual decision of each masked
//             problem from st[j].rho_new = ||b - A x||^2: DONE, MAXIT,
//             BREAKDOWN (DONE stamps the device clock: the problem's
//             latency ends there), or a residual replacement that restarts the
//             recurrence (beta = ||r||^2 / rho, rho = rmax2 = ||r||^2; the
//             problem rejoins the active count and is marked for p = r + beta p)
__global__ void __launch_bounds__(FIN_BLOCK) batch_finalize_kernel(BatchArgs a, int mode, double *bnorm2) {
    if ((mode == FIN_PQ || mode == FIN_XR) && *a.nactive == 0)
        return;
    const int j = blockIdx.x * (FIN_BLOCK / 64) + (threadIdx.x >> 6);
    if (j >= a.nprob)  // uniform over the wavefront
        return;
    if (mode == FIN_RESTART) {
        if ((threadIdx.x & 63) != 0)
            return;
        CgScalars s = a.st[j];
        s.restart = 0;
        if (a.mask[j]) {
            const double r2 = s.rho_new;
            a.mask[j] = 0;
            s.rtrue2 = r2;
            if (!(r2 >= 0.0 && r2 < 1.0e308)) {
                s.flag = FLAG_BREAKDOWN;
            } else if (r2 <= s.target2) {
                s.flag = FLAG_DONE;
                // the solve ends here, when its FP64 true residual confirms it
                s.spare = (double)wall_clock64();
            } else if (s.iters >= s.max_iter) {
                s.flag = FLAG_MAXIT;
            } else {
                s.nrel += 1;
                s.beta = r2 / s.rho;
                s.rho = r2;
                s.rmax2 = r2;
                s.flag = FLAG_RUN;
                s.active = 1;
                s.restart = 1;
                atomicAdd(a.nactive, 1);
            }
        }
        a.st[j] = s;
        if (j == 0)
            *a.npend = 0;  // read by later launches only
        return;
    }
    const BatchProb &P = a.probs[j];
    const double tot = wave_sum_slot(a.partials + P.first_blk, P.nblk);
    if ((threadIdx.x & 63) != 0)
        return;
    if (mode == FIN_BNORM) {
        bnorm2[j] = tot;
        return;
    }
    if (mode == FIN_RESID) {
        if (a.mask[j])
            a.st[j].rho_new = tot;
        return;
    }
    CgScalars s = a.st[j];
    if (!s.active)
        return;
    if (mode == FIN_PQ) {
        a.st[j].pq = tot;
        return;
    }
    if (!pos_finite(s.pq)) {
        s.flag = FLAG_BREAKDOWN;
        s.active = 0;
    } else {
        const double rho_new = tot;
        s.iters += 1;
        s.rho_new = rho_new;
        if (!(rho_new == rho_new)) {
            s.flag = FLAG_BREAKDOWN;
            s.active = 0;
        } else if (rho_new <= s.target2) {
            s.flag = FLAG_CONV;
            s.active = 0;
            a.mask[j] = 1;  // true residual at the next check
            *a.npend = 1;
        } else if (s.delta2 > 0.0 && rho_new < s.delta2 * s.rmax2) {
            s.flag = FLAG_RELIABLE;
            s.active = 0;
            a.mask[j] = 1;
            *a.npend = 1;
        } else if (s.iters >= s.max_iter) {
            s.flag = FLAG_MAXIT;
            s.active = 0;
        } else {
            s.beta = rho_new / s.rho;
            s.rho = rho_new;
            s.rmax2 = fmax(s.rmax2, rho_new);
        }
    }
    if (!s.active) {
        s.spare = (double)wall_clock64();  // device clock when the recurrence stopped
        atomicSub(a.nactive, 1);
    }
    a.st[j] = s;
}

// p = r + beta p for active problems (RESTART: for the problems the last
// true-residual decision restarted).
template <int FP, int TB, bool RESTART>
__global__ void __launch_bounds__(TB) batch_p_kernel(BatchArgs a) {
    using T = typename SloppyT<FP>::T;
    if (*a.nactive == 0)
        return;
    const int blk = blockIdx.x;
    const int j = a.blk_prob[blk];
    const BatchProb &P = a.probs[j];
    const int i = (blk - P.first_blk) * TB + threadIdx.x;
    const CgScalars st = a.st[j];
    if (!(RESTART ? st.restart : st.active) || i >= P.g.vh)
        return;
    cplx<T> p[3], r[3];
    FieldIO<FP>::template load<T>(P.p, P.g.vh, 1, 0, i, p);
    FieldIO<FP>::template load<T>(P.r, P.g.vh, 1, 0, i, r);
    const T b = (T)st.beta;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        p[c].re = fma(b, p[c].re, r[c].re);
        p[c].im = fma(b, p[c].im, r[c].im);
    }
    FieldIO<FP>::template store<T>(P.p, P.g.vh, 1, 0, i, p);
}

// For masked problems: r = b - ax (sloppy copy) and block partials of
// ||b - ax||^2 (FP64); with `copy_p` also p = r (start of a solve).
template <int FP, int TB>
__global__ void __launch_bounds__(TB) batch_residual_kernel(BatchArgs a, int copy_p) {
    using T = typename SloppyT<FP>::T;
    if (*a.npend == 0)
        return;
    const int blk = blockIdx.x;
    const int j = a.blk_prob[blk];
    const BatchProb &P = a.probs[j];
    const int i = (blk - P.first_blk) * TB + threadIdx.x;
    double part[1] = {0.0};
    if (a.mask[j] && i < P.g.vh) {
        cplx<double> bv[3], av[3];
        FieldIO<HISQ_FP64>::template load<double>(P.b, P.g.vh, 1, 0, i, bv);
        FieldIO<HISQ_FP64>::template load<double>(P.ax, P.g.vh, 1, 0, i, av);
        cplx<T> rv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double re = bv[c].re - av[c].re, im = bv[c].im - av[c].im;
            part[0] = fma(re, re, part[0]);
            part[0] = fma(im, im, part[0]);
            rv[c].re = (T)re;
            rv[c].im = (T)im;
        }
        FieldIO<FP>::template store<T>(P.r, P.g.vh, 1, 0, i, rv);
        if (copy_p)
            FieldIO<FP>::template store<T>(P.p, P.g.vh, 1, 0, i, rv);
    }
    __shared__ double lds[TB / 64];
    block_sum<1>(part, lds);
    if (threadIdx.x == 0)
        a.partials[blk] = part[0];
}

// Block partials of ||b||^2 of every problem (used once, before the solve).
template <int TB>
__global__ void __launch_bounds__(TB) batch_bnorm_kernel(BatchArgs a) {
    const int blk = blockIdx.x;
    const int j = a.blk_prob[blk];
    const BatchProb &P = a.probs[j];
    const int i = (blk - P.first_blk) * TB + threadIdx.x;
    double part[1] = {0.0};
    if (i < P.g.vh) {
        cplx<double> bv[3];
        FieldIO<HISQ_FP64>::template load<double>(P.b, P.g.vh, 1, 0, i, bv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            part[0] = fma(bv[c].re, bv[c].re, part[0]);
            part[0] = fma(bv[c].im, bv[c].im, part[0]);
        }
    }
    __shared__ double lds[TB / 64];
    block_sum<1>(part, lds);
    if (threadIdx.x == 0)
        a.partials[blk] = part[0];
}

__global__ void batch_clock_kernel(double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *out = (double)wall_clock64();
}

template <int TB>
hipError_t launch_batch_tb(const BatchArgs &a, int nblocks, int op, int lp, hipStream_t st) {
    const dim3 g((unsigned)nblocks);
    const bool f64 = lp == HISQ_FP64;
    const bool f16 = lp == HISQ_FP16N;
    switch (op) {
    case BOP_ITER_DOE:
        if (f64) batch_dslash_kernel<HISQ_FP64, HISQ_FP64, ROLE_ITER_DOE, TB><<<g, TB, 0, st>>>(a);
        else if (f16) batch_dslash_kernel<HISQ_FP16N, HISQ_FP32, ROLE_ITER_DOE, TB><<<g, TB, 0, st>>>(a);
        else batch_dslash_kernel<HISQ_FP32, HISQ_FP32, ROLE_ITER_DOE, TB><<<g, TB, 0, st>>>(a);
        break;
    case BOP_ITER_DEO:
        if (f64) batch_dslash_kernel<HISQ_FP64, HISQ_FP64, ROLE_ITER_DEO, TB><<<g, TB, 0, st>>>(a);
        else if (f16) batch_dslash_kernel<HISQ_FP16N, HISQ_FP32, ROLE_ITER_DEO, TB><<<g, TB, 0, st>>>(a);
        else batch_dslash_kernel<HISQ_FP32, HISQ_FP32, ROLE_ITER_DEO, TB><<<g, TB, 0, st>>>(a);
        break;
    case BOP_TRUE_DOE: batch_dslash_kernel<HISQ_FP64, HISQ_FP64, ROLE_TRUE_DOE, TB><<<g, TB, 0, st>>>(a); break;
    case BOP_TRUE_DEO: batch_dslash_kernel<HISQ_FP64, HISQ_FP64, ROLE_TRUE_DEO, TB><<<g, TB, 0, st>>>(a); break;
    case BOP_XR:
        if (f64) batch_xr_kernel<HISQ_FP64, TB><<<g, TB, 0, st>>>(a);
        else batch_xr_kernel<HISQ_FP32, TB><<<g, TB, 0, st>>>(a);
        break;
    case BOP_P:
        if (f64) batch_p_kernel<HISQ_FP64, TB, false><<<g, TB, 0, st>>>(a);
        else batch_p_kernel<HISQ_FP32, TB, false><<<g, TB, 0, st>>>(a);
        break;
    case BOP_RESTART:
        if (f64) batch_p_kernel<HISQ_FP64, TB, true><<<g, TB, 0, st>>>(a);
        else batch_p_kernel<HISQ_FP32, TB, true><<<g, TB, 0, st>>>(a);
        break;
    case BOP_RESIDUAL:
    case BOP_RESIDUAL_COPY_P: {
        const int cp = op == BOP_RESIDUAL_COPY_P;
        if (f64) batch_residual_kernel<HISQ_FP64, TB><<<g, TB, 0, st>>>(a, cp);
        else batch_residual_kernel<HISQ_FP32, TB><<<g, TB, 0, st>>>(a, cp);
        break;
    }
    case BOP_BNORM: batch_bnorm_kernel<TB><<<g, TB, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_batch(const BatchArgs &a, int nblocks, int op, int lp, hipStream_t st) {
    if (op == BOP_RESTART) {
        batch_finalize_kernel<<<(a.nprob + 3) / 4, FIN_BLOCK, 0, st>>>(a, FIN_RESTART, nullptr);
        const hipError_t e0 = hipGetLastError();
        if (e0 != hipSuccess)
            return e0;
    }
    hipError_t e = a.block == 64    ? launch_batch_tb<64>(a, nblocks, op, lp, st)
                   : a.block == 128 ? launch_batch_tb<128>(a, nblocks, op, lp, st)
                   : a.block == 256 ? launch_batch_tb<256>(a, nblocks, op, lp, st)
                                    : hipErrorInvalidValue;
    if (e != hipSuccess)
        return e;
    const int fin = op == BOP_ITER_DEO ? FIN_PQ : op == BOP_XR ? FIN_XR
                    : (op == BOP_RESIDUAL || op == BOP_RESIDUAL_COPY_P) ? FIN_RESID : -1;
    if (fin < 0)
        return hipSuccess;
    batch_finalize_kernel<<<(a.nprob + 3) / 4, FIN_BLOCK, 0, st>>>(a, fin, nullptr);
    return hipGetLastError();
}

hipError_t launch_batch_bnorm(const BatchArgs &a, int nblocks, double *bnorm2, hipStream_t st) {
    hipError_t e = a.block == 64    ? launch_batch_tb<64>(a, nblocks, BOP_BNORM, HISQ_FP64, st)
                   : a.block == 128 ? launch_batch_tb<128>(a, nblocks, BOP_BNORM, HISQ_FP64, st)
                   : a.block == 256 ? launch_batch_tb<256>(a, nblocks, BOP_BNORM, HISQ_FP64, st)
                                    : hipErrorInvalidValue;
    if (e != hipSuccess)
        return e;
    batch_finalize_kernel<<<(a.nprob + 3) / 4, FIN_BLOCK, 0, st>>>(a, FIN_BNORM, bnorm2);
    return hipGetLastError();
}

hipError_t launch_batch_clock(double *out, hipStream_t st) {
    batch_clock_kernel<<<1, 64, 0, st>>>(out);
    return hipGetLastError();
}

}  // namespace hisq
