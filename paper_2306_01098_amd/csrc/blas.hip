// Vector kernels of the CG family: fused solution/residual updates with the
// residual norm, direction updates, true-residual formation, norms, copies.
// Reductions are FP64 and deterministic (block partials, then a one-block
// finalize); the Krylov scalars are advanced in FP64 by the finalize kernel.
#include "internal.hpp"
#include "reduce.hpp"
#include "solver.hpp"

namespace hisq {

namespace {

constexpr int BLK = 256;

template <int FP> struct Sloppy;
template <> struct Sloppy<HISQ_FP64> { using T = double; };
template <> struct Sloppy<HISQ_FP32> { using T = float; };

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v < 1.0e308; }

// <p, A p> of column rr from the D_eo kernel's block partials: wave 0 sums
// them (wave_sum_slot: the order cg_finalize_kernel uses too) and the block
// reads the total from LDS.
__device__ __forceinline__ double block_pq(const CgVecParams &prm, int rr, double *lds1) {
    if (threadIdx.x < 64) {
        const double v = wave_sum_slot<false>(prm.pq_part + (size_t)rr * prm.pq_nblk, prm.pq_nblk);
        if (threadIdx.x == 0)
            *lds1 = v;
    }
    __syncthreads();
    return *lds1;
}

// x += alpha p (FP64 x), r -= alpha q with alpha = rho / <p, A p>, and the
// block partials of <r, r> for right-hand side blockIdx.y; multi-shift:
// x_k += alpha_k p_k.
template <int FP>
__global__ void __launch_bounds__(BLK) cg_xr_kernel(CgVecParams prm) {
    using T = typename Sloppy<FP>::T;
    if (*prm.skip)
        return;
    __shared__ double lds[4];
    __shared__ double pq_s;
    const int rr = blockIdx.y;
    const int i = blockIdx.x * BLK + threadIdx.x;
    const CgScalars st = prm.st[rr];
    const bool mine = st.active && i < prm.vh;
    cplx<T> p[3], q[3], r[3];
    cplx<double> x[3];
    if (mine) {  // issued before the <p, A p> sum so the loads overlap it
        FieldIO<FP>::template load<T>(prm.p, prm.vh, rr, i, p);
        FieldIO<FP>::template load<T>(prm.q, prm.vh, rr, i, q);
        FieldIO<FP>::template load<T>(prm.r, prm.vh, rr, i, r);
        FieldIO<HISQ_FP64>::template load<double>(prm.x[rr], prm.vh, 0, i, x);
    }
    const double pq = block_pq(prm, rr, &pq_s);
    const bool go = st.active && finite_pos(pq);
    const double alpha = go ? st.rho / pq : 0.0;
    double part[1] = {0.0};
    if (go && mine) {
        const T a = (T)alpha;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[c].re = fma(alpha, (double)p[c].re, x[c].re);
            x[c].im = fma(alpha, (double)p[c].im, x[c].im);
            r[c].re = fma(-a, q[c].re, r[c].re);
            r[c].im = fma(-a, q[c].im, r[c].im);
            part[0] = fma((double)r[c].re, (double)r[c].re, part[0]);
            part[0] = fma((double)r[c].im, (double)r[c].im, part[0]);
        }
        FieldIO<HISQ_FP64>::template store<double>(prm.x[rr], prm.vh, 0, i, x);
        FieldIO<FP>::template store<T>(prm.r, prm.vh, rr, i, r);
        if (prm.nshift > 0) {
            // shifted solutions: alpha_k = alpha zeta_new / zeta (Jegerlehner)
            const MsGlobal ms = *prm.ms;
            for (int k = 0; k < prm.nshift; ++k) {
                const ShiftScalars sk = prm.sh[k];
                if (!sk.active)
                    continue;
                const double den = alpha * ms.beta_old * (sk.zeta_old - sk.zeta) +
                                   sk.zeta_old * ms.alpha_old * (1.0 + sk.s * alpha);
                const double zn = sk.zeta * sk.zeta_old * ms.alpha_old / den;
                const double ak = alpha * zn / sk.zeta;
                cplx<T> pk[3];
                cplx<double> xk[3];
                FieldIO<FP>::template load<T>(prm.ps, prm.vh, k, i, pk);
                FieldIO<HISQ_FP64>::template load<double>(prm.xs[k], prm.vh, 0, i, xk);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xk[c].re = fma(ak, (double)pk[c].re, xk[c].re);
                    xk[c].im = fma(ak, (double)pk[c].im, xk[c].im);
                }
                FieldIO<HISQ_FP64>::template store<double>(prm.xs[k], prm.vh, 0, i, xk);
            }
        }
    }
    block_sum<1>(part, lds);
    if (threadIdx.x == 0)
        prm.partials[(size_t)rr * gridDim.x + blockIdx.x] = part[0];
}

// One block: sums the <r, r> partials of cg_xr_kernel (nblk blocks per
// right-hand side) and the <p, A p> partials of the D_eo kernel (in the order
// cg_xr_kernel summed them) and advances the scalars: breakdown check, rho, beta,
// convergence / reliable-update / iteration-limit flags, and the multi-shift
// zeta recurrences.
__global__ void __launch_bounds__(1024) cg_finalize_kernel(CgVecParams prm, int nblk) {
    if (*prm.skip)
        return;
    __shared__ double tot[HISQ_MAX_RHS];
    __shared__ double totpq[HISQ_MAX_RHS];
    sum_partials_block(prm.partials, prm.nrhs, nblk, tot);
    for (int j = threadIdx.x >> 6; j < prm.nrhs; j += blockDim.x >> 6) {
        const double v = wave_sum_slot<false>(prm.pq_part + (size_t)j * prm.pq_nblk, prm.pq_nblk);
        if ((threadIdx.x & 63) == 0)
            totpq[j] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0)
        return;
    int any = 0;
    for (int j = 0; j < prm.nrhs; ++j) {
        CgScalars s = prm.st[j];
        if (s.active) {
            s.pq = totpq[j];
            if (!finite_pos(s.pq)) {
                s.flag = FLAG_BREAKDOWN;
                s.active = 0;
            } else {
                const double a = s.rho / s.pq;
                const double rho_new = tot[j];
                s.iters += 1;
                s.rho_new = rho_new;
                if (j == 0 && prm.nshift > 0) {
                    // advance the shifted systems before beta is formed
                    const double beta = rho_new / s.rho;
                    MsGlobal ms = *prm.ms;
                    for (int k = 0; k < prm.nshift; ++k) {
                        ShiftScalars sk = prm.sh[k];
                        if (!sk.active)
                            continue;
                        const double den = a * ms.beta_old * (sk.zeta_old - sk.zeta) +
                                           sk.zeta_old * ms.alpha_old * (1.0 + sk.s * a);
                        const double zn = sk.zeta * sk.zeta_old * ms.alpha_old / den;
                        sk.alpha = a * zn / sk.zeta;
                        sk.beta = beta * (zn / sk.zeta) * (zn / sk.zeta);
                        sk.zeta_old = sk.zeta;
                        sk.zeta = zn;
                        sk.zeta_new = zn;
                        sk.iters = s.iters;
                        if (!(zn == zn) || zn * zn * rho_new <= sk.target2) {
                            sk.active = 0;  // converged (or underflowed): frozen
                            sk.flag = FLAG_CONV;
                        }
                        prm.sh[k] = sk;
                    }
                    ms.alpha_old = a;
                    ms.beta_old = beta;
                    *prm.ms = ms;
                }
                if (!(rho_new == rho_new)) {
                    s.flag = FLAG_BREAKDOWN;
                    s.active = 0;
                } else if (rho_new <= s.target2) {
                    s.flag = FLAG_CONV;
                    s.active = 0;
                    prm.tr_skip[j] = 0;
                    if (prm.nopend)
                        *prm.nopend = 0;
                } else if (s.delta2 > 0.0 && rho_new < s.delta2 * s.rmax2) {
                    s.flag = FLAG_RELIABLE;
                    s.active = 0;
                    prm.tr_skip[j] = 0;
                    if (prm.nopend)
                        *prm.nopend = 0;
                } else if (s.iters >= s.max_iter) {
                    s.flag = FLAG_MAXIT;
                    s.active = 0;
                } else {
                    s.beta = rho_new / s.rho;
                    s.rho = rho_new;
                    s.rmax2 = fmax(s.rmax2, rho_new);
                }
            }
            prm.st[j] = s;
        }
        any |= s.active;
    }
    *prm.skip = any ? 0 : 1;
}

// The true-residual check of the columns that raised FLAG_CONV or
// FLAG_RELIABLE (tr_skip[j] == 0), after r_j = b_j - A x_j and the block
// partials of ||r_j||^2 (nblk per column in trpart) were formed: the FP64
// norm decides DONE (target met), MAXIT, or a residual replacement, which
// restarts the recurrence with beta = ||r||^2 / rho, rho = rmax2 = ||r||^2
// (p = r + beta p follows in cg_p_kernel's restart mode).  One block.
__global__ void __launch_bounds__(1024) cg_restart_kernel(CgVecParams prm, const double *trpart, int nblk) {
    __shared__ double tot[HISQ_MAX_RHS];
    for (int j = threadIdx.x >> 6; j < prm.nrhs; j += blockDim.x >> 6)
        if (prm.tr_skip[j] == 0) {
            const double v = wave_sum_slot<true>(trpart + (size_t)j * nblk, nblk);
            if ((threadIdx.x & 63) == 0)
                tot[j] = v;
        }
    __syncthreads();
    if (threadIdx.x != 0)
        return;
    int any = 0;
    for (int j = 0; j < prm.nrhs; ++j) {
        CgScalars s = prm.st[j];
        s.restart = 0;
        if (prm.tr_skip[j] == 0) {
            const double r2 = tot[j];
            prm.tr_skip[j] = 1;
            s.rtrue2 = r2;
            if (!(r2 >= 0.0 && r2 < 1.0e308)) {
                s.flag = FLAG_BREAKDOWN;
                s.active = 0;
            } else if (r2 <= s.target2) {
                s.flag = FLAG_DONE;
                s.active = 0;
            } else if (s.iters >= s.max_iter) {
                s.flag = FLAG_MAXIT;
                s.active = 0;
            } else {
                s.nrel += 1;
                s.beta = r2 / s.rho;
                s.rho = r2;
                s.rmax2 = r2;
                s.flag = FLAG_RUN;
                s.active = 1;
                s.restart = 1;
            }
        }
        prm.st[j] = s;
        any |= s.active;
    }
    *prm.skip = any ? 0 : 1;
    if (prm.nopend)
        *prm.nopend = 1;
}

// p = r + beta p for right-hand side rhs0 + blockIdx.y (if active; in restart
// mode only for a column just restarted by cg_restart_kernel);
// multi-shift: p_k = zeta_k r + beta_k p_k.
template <int FP>
__global__ void __launch_bounds__(BLK) cg_p_kernel(CgVecParams prm, int rhs0, int restart_only) {
    using T = typename Sloppy<FP>::T;
    if (*prm.skip)
        return;
    const int rr = rhs0 + blockIdx.y;
    const int i = blockIdx.x * BLK + threadIdx.x;
    const CgScalars st = prm.st[rr];
    if (!(restart_only ? st.restart : st.active) || i >= prm.vh)
        return;
    cplx<T> p[3], r[3];
    FieldIO<FP>::template load<T>(prm.p, prm.vh, rr, i, p);
    FieldIO<FP>::template load<T>(prm.r, prm.vh, rr, i, r);
    const T b = (T)st.beta;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        p[c].re = fma(b, p[c].re, r[c].re);
        p[c].im = fma(b, p[c].im, r[c].im);
    }
    FieldIO<FP>::template store<T>(prm.p, prm.vh, rr, i, p);
    if (prm.nshift > 0 && rr == 0) {
        for (int k = 0; k < prm.nshift; ++k) {
            const ShiftScalars sk = prm.sh[k];
            if (!sk.active)
                continue;
            cplx<T> pk[3];
            FieldIO<FP>::template load<T>(prm.ps, prm.vh, k, i, pk);
            const T z = (T)sk.zeta, bk = (T)sk.beta;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pk[c].re = fma(bk, pk[c].re, z * r[c].re);
                pk[c].im = fma(bk, pk[c].im, z * r[c].im);
            }
            FieldIO<FP>::template store<T>(prm.ps, prm.vh, k, i, pk);
        }
    }
}

// r = b - ax (FP64 inputs; r stored in the sloppy precision) and
// *out2 = ||b - ax||^2 in FP64 (from the FP64 values).
template <int FP>
__global__ void __launch_bounds__(BLK) residual_kernel(int vh, const void *b, const void *ax, void *r,
                                                       double *partials, const int *skip) {
    using T = typename Sloppy<FP>::T;
    if (skip && *skip)
        return;
    __shared__ double lds[4];
    const int i = blockIdx.x * BLK + threadIdx.x;
    double part[1] = {0.0};
    if (i < vh) {
        cplx<double> bv[3], av[3];
        FieldIO<HISQ_FP64>::template load<double>(b, vh, 0, i, bv);
        FieldIO<HISQ_FP64>::template load<double>(ax, vh, 0, i, av);
        cplx<T> rv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double re = bv[c].re - av[c].re, im = bv[c].im - av[c].im;
            part[0] = fma(re, re, part[0]);
            part[0] = fma(im, im, part[0]);
            rv[c].re = (T)re;
            rv[c].im = (T)im;
        }
        FieldIO<FP>::template store<T>(r, vh, 0, i, rv);
    }
    block_sum<1>(part, lds);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = part[0];
}

// Block partials of ||v||^2 of an FP64 field (one column).
__global__ void __launch_bounds__(BLK) norm2_kernel(int vh, const void *v, double *partials) {
    __shared__ double lds[4];
    const int i = blockIdx.x * BLK + threadIdx.x;
    double part[1] = {0.0};
    if (i < vh) {
        cplx<double> a[3];
        FieldIO<HISQ_FP64>::template load<double>(v, vh, 0, i, a);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            part[0] = fma(a[c].re, a[c].re, part[0]);
            part[0] = fma(a[c].im, a[c].im, part[0]);
        }
    }
    block_sum<1>(part, lds);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = part[0];
}

// Block partials of Re <a_r, b_r> for FP64 fields, column r = blockIdx.y.
__global__ void __launch_bounds__(BLK) dot_re_kernel(int vh, const void *a, const void *b, double *partials) {
    __shared__ double lds[4];
    const int r = blockIdx.y;
    const int i = blockIdx.x * BLK + threadIdx.x;
    double part[1] = {0.0};
    if (i < vh) {
        cplx<double> u[3], v[3];
        FieldIO<HISQ_FP64>::template load<double>(a, vh, r, i, u);
        FieldIO<HISQ_FP64>::template load<double>(b, vh, r, i, v);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            part[0] = fma(u[c].re, v[c].re, part[0]);
            part[0] = fma(u[c].im, v[c].im, part[0]);
        }
    }
    block_sum<1>(part, lds);
    if (threadIdx.x == 0)
        partials[(size_t)r * gridDim.x + blockIdx.x] = part[0];
}

// dst = src for n fields, with precision conversion.
template <int FS, int FD>
__global__ void __launch_bounds__(BLK) copy_kernel(int vh, int n, const void *src, void *dst) {
    using T = typename Sloppy<FD>::T;
    const int i = blockIdx.x * BLK + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= vh || r >= n)
        return;
    cplx<T> v[3];
    FieldIO<FS>::template load<T>(src, vh, r, i, v);
    FieldIO<FD>::template store<T>(dst, vh, r, i, v);
}

__global__ void __launch_bounds__(BLK) fill_u32_kernel(unsigned *p, size_t n, unsigned v) {
    const size_t i = (size_t)blockIdx.x * BLK + threadIdx.x;
    if (i < n)
        p[i] = v;
}

inline dim3 grid_for(int vh, int ny = 1) { return dim3((unsigned)((vh + BLK - 1) / BLK), (unsigned)ny); }

}  // namespace

int blas_blocks(int vh) { return (vh + BLK - 1) / BLK; }

hipError_t launch_cg_xr(const CgVecParams &p, int fp, hipStream_t st) {
    const dim3 g = grid_for(p.vh, p.nrhs);
    if (fp == HISQ_FP64)
        cg_xr_kernel<HISQ_FP64><<<g, BLK, 0, st>>>(p);
    else
        cg_xr_kernel<HISQ_FP32><<<g, BLK, 0, st>>>(p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    cg_finalize_kernel<<<1, 1024, 0, st>>>(p, (int)g.x);
    return hipGetLastError();
}

hipError_t launch_cg_p(const CgVecParams &p, int fp, int rhs0, int nrhs, hipStream_t st, bool restart_only) {
    const int mode = restart_only ? 1 : 0;
    if (fp == HISQ_FP64)
        cg_p_kernel<HISQ_FP64><<<grid_for(p.vh, nrhs), BLK, 0, st>>>(p, rhs0, mode);
    else
        cg_p_kernel<HISQ_FP32><<<grid_for(p.vh, nrhs), BLK, 0, st>>>(p, rhs0, mode);
    return hipGetLastError();
}

hipError_t launch_cg_restart(const CgVecParams &p, const double *trpart, hipStream_t st) {
    cg_restart_kernel<<<1, 1024, 0, st>>>(p, trpart, blas_blocks(p.vh));
    return hipGetLastError();
}

hipError_t launch_residual_parts(int vh, int fp, const void *b, const void *ax, void *r, double *partials,
                                 const int *skip, hipStream_t st) {
    if (fp == HISQ_FP64)
        residual_kernel<HISQ_FP64><<<grid_for(vh), BLK, 0, st>>>(vh, b, ax, r, partials, skip);
    else
        residual_kernel<HISQ_FP32><<<grid_for(vh), BLK, 0, st>>>(vh, b, ax, r, partials, skip);
    return hipGetLastError();
}

hipError_t launch_residual(int vh, int fp, const void *b, const void *ax, void *r, double *partials,
                           double *out2, hipStream_t st) {
    hipError_t e = launch_residual_parts(vh, fp, b, ax, r, partials, nullptr, st);
    return e == hipSuccess ? launch_sum_partials(partials, 1, blas_blocks(vh), out2, 1, nullptr, st) : e;
}

hipError_t launch_norm2(int vh, const void *v, double *partials, double *out2, hipStream_t st) {
    norm2_kernel<<<grid_for(vh), BLK, 0, st>>>(vh, v, partials);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? launch_sum_partials(partials, 1, blas_blocks(vh), out2, 1, nullptr, st) : e;
}

hipError_t launch_dot_re(int vh, int n, const void *a, const void *b, double *partials, double *out, hipStream_t st) {
    dot_re_kernel<<<grid_for(vh, n), BLK, 0, st>>>(vh, a, b, partials);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? launch_sum_partials(partials, n, blas_blocks(vh), out, 1, nullptr, st) : e;
}

hipError_t launch_copy(int vh, int n, int fs, int fd, const void *src, void *dst, hipStream_t st) {
    const dim3 g = grid_for(vh, n);
    if (fs == HISQ_FP64 && fd == HISQ_FP64)
        copy_kernel<HISQ_FP64, HISQ_FP64><<<g, BLK, 0, st>>>(vh, n, src, dst);
    else if (fs == HISQ_FP64 && fd == HISQ_FP32)
        copy_kernel<HISQ_FP64, HISQ_FP32><<<g, BLK, 0, st>>>(vh, n, src, dst);
    else if (fs == HISQ_FP32 && fd == HISQ_FP32)
        copy_kernel<HISQ_FP32, HISQ_FP32><<<g, BLK, 0, st>>>(vh, n, src, dst);
    else if (fs == HISQ_FP32 && fd == HISQ_FP64)
        copy_kernel<HISQ_FP32, HISQ_FP64><<<g, BLK, 0, st>>>(vh, n, src, dst);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t st) {
    if (n == 0)
        return hipSuccess;
    fill_u32_kernel<<<dim3((unsigned)((n + BLK - 1) / BLK)), BLK, 0, st>>>(p, n, v);
    return hipGetLastError();
}

}  // namespace hisq
