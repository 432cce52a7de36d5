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
        FieldIO<FP>::template load<T>(prm.p, prm.vh, prm.nrhs, rr, i, p);
        FieldIO<FP>::template load<T>(prm.q, prm.vh, prm.nrhs, rr, i, q);
        FieldIO<FP>::template load<T>(prm.r, prm.vh, prm.nrhs, rr, i, r);
        FieldIO<HISQ_FP64>::template load<double>(prm.x[rr], prm.vh, 1, 0, i, x);
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
        FieldIO<HISQ_FP64>::template store<double>(prm.x[rr], prm.vh, 1, 0, i, x);
        FieldIO<FP>::template store<T>(prm.r, prm.vh, prm.nrhs, rr, i, r);
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
                FieldIO<FP>::template load<T>(prm.ps, prm.vh, 1, k, i, pk);
                FieldIO<HISQ_FP64>::template load<double>(prm.xs[k], prm.vh, 1, 0, i, xk);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xk[c].re = fma(ak, (double)pk[c].re, xk[c].re);
                    xk[c].im = fma(ak, (double)pk[c].im, xk[c].im);
                }
                FieldIO<HISQ_FP64>::template store<double>(prm.xs[k], prm.vh, 1, 0, i, xk);
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
    FieldIO<FP>::template load<T>(prm.p, prm.vh, prm.nrhs, rr, i, p);
    FieldIO<FP>::template load<T>(prm.r, prm.vh, prm.nrhs, rr, i, r);
    const T b = (T)st.beta;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        p[c].re = fma(b, p[c].re, r[c].re);
        p[c].im = fma(b, p[c].im, r[c].im);
    }
    FieldIO<FP>::template store<T>(prm.p, prm.vh, prm.nrhs, rr, i, p);
    if (prm.nshift > 0 && rr == 0) {
        for (int k = 0; k < prm.nshift; ++k) {
            const ShiftScalars sk = prm.sh[k];
            if (!sk.active)
                continue;
            cplx<T> pk[3];
            FieldIO<FP>::template load<T>(prm.ps, prm.vh, 1, k, i, pk);
            const T z = (T)sk.zeta, bk = (T)sk.beta;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pk[c].re = fma(bk, pk[c].re, z * r[c].re);
                pk[c].im = fma(bk, pk[c].im, z * r[c].im);
            }
            FieldIO<FP>::template store<T>(prm.ps, prm.vh, 1, k, i, pk);
        }
    }
}

// ---------------------------------------------------------------------------
// Single-reduction CG (after Chronopoulos and Gear).  With w = A r formed by
// the D_eo kernel together with the block partials of Re <r, w>, one scalar
// step per iteration needs all inner products at once:
//   gamma = <r, r>,  delta = Re <r, w>,  beta = gamma / gamma_old,
//   <p_new, A p_new> = <r + beta p, w + beta s>
//                    = delta + beta (2 Re <r, s> + beta <p, s>),
//   alpha = gamma / <p_new, A p_new>,
//   p = r + beta p,  s = w + beta s (= A p),  x += alpha p,  r -= alpha s,
// where <r, r>, Re <r, s> and <p, s> of the new vectors are summed by the
// same update kernel.  (Chronopoulos and Gear write <p, A p> as
// delta - beta gamma / alpha_old, which assumes r _|_ r_old and s = A p
// exactly; with FP16 links that form lost all accuracy after a few hundred
// iterations, CPU emulation: <p, A p> = -0.41 where the direct value is 7.9.)
// In exact arithmetic these are the iterates of the Hestenes-Stiefel CG; the
// launches per iteration drop from five to four (D_oe, D_eo, scalars, update).
// ---------------------------------------------------------------------------

// The scalar step of one column from the sums tot = {<r, r>, Re <r, w>,
// Re <r, s>, <p, s>} of its partials.  decide: the check block has just formed
// the column's FP64 true residual (it waited for it), so ||b - A x||^2 is in
// tot[0] (and Re <r, s> of the replaced r in tot[2]) and the column is decided
// first: done, the iteration limit, or a residual replacement (the reliable
// update of Clark et al.), after which the same step continues from the
// replaced r with beta = ||r||^2 / rho, as the two-reduction solver does.
// Sets s.go (0: no update; 1: update; 2: update with fresh directions).
// *wait: 1 when the column starts waiting for its true residual, 0 when it
// stopped waiting, unchanged otherwise.
__device__ __forceinline__ void cgcg_decide(CgScalars &s, const double (&tot)[4], bool decide, int *wait) {
    s.go = 0;
    const double gamma = tot[0], delta = tot[1];
    if (decide) {
        *wait = 0;
        s.rtrue2 = gamma;
        if (!(gamma >= 0.0 && gamma < 1.0e308)) {
            s.flag = FLAG_BREAKDOWN;
        } else if (gamma <= s.target2) {
            s.flag = FLAG_DONE;
        } else if (s.iters >= s.max_iter) {
            s.flag = FLAG_MAXIT;
        } else {
            s.nrel += 1;
            s.rmax2 = gamma;
            s.flag = FLAG_RUN;
            s.active = 1;
        }
    }
    if (!s.active)
        return;
    if (!(gamma >= 0.0 && gamma < 1.0e308) || !(delta == delta)) {
        s.flag = FLAG_BREAKDOWN;
        s.active = 0;
    } else if (gamma <= s.target2) {
        s.flag = FLAG_CONV;
        s.active = 0;
        *wait = 1;
    } else if (s.delta2 > 0.0 && gamma < s.delta2 * s.rmax2) {
        s.flag = FLAG_RELIABLE;
        s.active = 0;
        *wait = 1;
    } else if (s.iters >= s.max_iter) {
        s.flag = FLAG_MAXIT;
        s.active = 0;
    } else {
        const bool fresh = s.restart != 0;
        const double beta = fresh ? 0.0 : gamma / s.rho;
        const double pap = fresh ? delta : delta + beta * (2.0 * tot[2] + beta * tot[3]);
        if (!finite_pos(pap)) {
            s.flag = FLAG_BREAKDOWN;
            s.active = 0;
        } else {
            s.alpha = gamma / pap;
            s.beta = beta;
            s.pq = pap;
            s.rho = gamma;
            s.rho_new = gamma;
            s.rmax2 = fmax(s.rmax2, gamma);
            s.iters += 1;
            s.restart = 0;
            s.go = fresh ? 2 : 1;
        }
    }
}

// The four partial slots of column j, summed by the four wavefronts of a block
// (one each, fixed order: deterministic) into tot; `off` selects the set of
// <r, r>, Re <r, s> and <p, s> partials.  NT: non-temporal loads (one
// reading block per column).
template <bool NT>
__device__ __forceinline__ void cgcg_sums(const CgVecParams &prm, int j, size_t off, double (&tot)[4],
                                          double *lds) {
    // slot k by wave k mod (waves of the block): any block of 64 .. 256 threads
    const int nwaves = blockDim.x >> 6;
    const size_t o = off + (size_t)j * prm.rr_nblk;
    for (int k = threadIdx.x >> 6; k < 4; k += nwaves) {
        const double *slot = k == 0   ? prm.rr_part + o
                             : k == 1 ? prm.rw_part + (size_t)j * prm.rw_nblk
                             : k == 2 ? prm.rs_part + o
                                      : prm.ps_part + o;
        const double v = wave_sum_slot<NT>(slot, k == 1 ? prm.rw_nblk : prm.rr_nblk);
        if ((threadIdx.x & 63) == 0)
            lds[k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k)
        tot[k] = lds[k];
}

// One block of four wavefronts per right-hand side j = blockIdx.x: the sums of
// the column's partials and its scalar step.  after_check != 0: the check
// block ran just before this iteration, so a waiting column (tr_skip == 0) is
// decided here.
__global__ void __launch_bounds__(256) cgcg_finalize_kernel(CgVecParams prm, int after_check) {
    if (*prm.skip)
        return;
    const int j = blockIdx.x;
    __shared__ double lds[4];
    double tot[4];
    cgcg_sums<true>(prm, j, 0, tot, lds);
    if (threadIdx.x != 0)
        return;
    CgScalars s = prm.st[j];
    int wait = -1;
    cgcg_decide(s, tot, after_check && prm.tr_skip[j] == 0, &wait);
    if (wait >= 0)
        prm.tr_skip[j] = wait ? 0 : 1;
    prm.st[j] = s;
}

// Thread -> (site, column) of the single-reduction vector kernels.  One
// column per block (PAIR = false): column col0 + blockIdx.y, one site per
// thread.  Column pairs (PAIR = true, for FP32 fields of several columns,
// whose columns 2j and 2j + 1 share 16-byte records): blocks of twice the
// threads over the same sites, block row blockIdx.y taking columns
// col0 + 2 blockIdx.y + {0, 1}; lane l of wave w serves site
// 32 (w & 1) + (l >> 1) of the block's 64-site group w >> 1 for the column
// l & 1, so the two lanes of a site read one whole record and the partials
// come out bitwise as with one column per block (block_sum_pair).
template <bool PAIR> struct VecPos {
    int j;  // column (relative to col0)
    int i;  // site
    __device__ __forceinline__ VecPos() {
        if constexpr (PAIR) {
            const int t = threadIdx.x, w = t >> 6;
            j = 2 * (int)blockIdx.y + (t & 1);
            i = blockIdx.x * (blockDim.x >> 1) + (w >> 1) * 64 + (w & 1) * 32 + ((t & 63) >> 1);
        } else {
            j = blockIdx.y;
            i = blockIdx.x * blockDim.x + threadIdx.x;
        }
    }
    // the thread that holds the block's sums for column j
    __device__ __forceinline__ bool leader() const { return PAIR ? threadIdx.x < 2 : threadIdx.x == 0; }
};

template <int NV, bool PAIR> __device__ __forceinline__ void vec_block_sum(double (&v)[NV], double *lds) {
    if constexpr (PAIR)
        block_sum_pair<NV>(v, lds);
    else
        block_sum<NV>(v, lds);
}

// LDS doubles of vec_block_sum for blocks of up to 2 BLK threads.
constexpr int vec_lds(int nv, bool pair) { return pair ? (2 * BLK / 128) * 64 * nv : (BLK / 64) * nv; }

// The vector step of the columns the finalize kernel stepped (go = 1; go = 2:
// fresh directions p = r, s = w):
//   p = r + beta p, s = w + beta s, x += alpha p (FP64 x), r -= alpha s,
// with the block partials of <r, r>, Re <r, s> and Re <p, s> of the new
// vectors (their stored values).
// Block (0, 0) also sets the launch flags of the following kernels: skip while
// no column is active (a column waiting for its true residual idles until the
// check block, whose residual kernel clears skip again so that the next
// iteration decides it), nopend while none is waiting.  (No other block of
// this launch reads them.)
template <int FP, bool PAIR>
__global__ void __launch_bounds__(PAIR ? 2 * BLK : BLK) cgcg_update_kernel(CgVecParams prm) {
    using T = typename Sloppy<FP>::T;
    const VecPos<PAIR> at;
    const int j = at.j;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        int run = 0, pend = 0;
        for (int k = 0; k < prm.nrhs; ++k) {
            run |= prm.st[k].active;
            pend |= prm.tr_skip[k] == 0 ? 1 : 0;
        }
        *prm.skip = run ? 0 : 1;
        if (prm.nopend)
            *prm.nopend = pend ? 0 : 1;
    }
    const bool col = j < prm.nrhs;
    CgScalars st{};
    if (col)
        st = prm.st[j];
    if (!PAIR && !st.go)
        return;  // the whole block belongs to column j
    __shared__ double lds[vec_lds(3, PAIR)];
    const int i = at.i;
    double part[3] = {0.0, 0.0, 0.0};
    if (st.go && i < prm.vh) {
        cplx<T> r[3], w[3], p[3], sv[3];
        cplx<double> x[3];
        FieldIO<FP>::template load<T>(prm.r, prm.vh, prm.nrhs, j, i, r);
        FieldIO<FP>::template load<T>(prm.w, prm.vh, prm.nrhs, j, i, w);
        FieldIO<HISQ_FP64>::template load<double>(prm.x[j], prm.vh, 1, 0, i, x);
        const bool fresh = st.go == 2;
        if (!fresh) {
            FieldIO<FP>::template load<T>(prm.p, prm.vh, prm.nrhs, j, i, p);
            FieldIO<FP>::template load<T>(prm.s, prm.vh, prm.nrhs, j, i, sv);
        }
        const T b = (T)st.beta, a = (T)st.alpha;
        const double ad = st.alpha;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (fresh) {
                p[c] = r[c];
                sv[c] = w[c];
            } else {
                p[c].re = fma(b, p[c].re, r[c].re);
                p[c].im = fma(b, p[c].im, r[c].im);
                sv[c].re = fma(b, sv[c].re, w[c].re);
                sv[c].im = fma(b, sv[c].im, w[c].im);
            }
            x[c].re = fma(ad, (double)p[c].re, x[c].re);
            x[c].im = fma(ad, (double)p[c].im, x[c].im);
            r[c].re = fma(-a, sv[c].re, r[c].re);
            r[c].im = fma(-a, sv[c].im, r[c].im);
            const double rre = r[c].re, rim = r[c].im, sre = sv[c].re, sim = sv[c].im;
            part[0] = fma(rre, rre, part[0]);
            part[0] = fma(rim, rim, part[0]);
            part[1] = fma(rre, sre, part[1]);
            part[1] = fma(rim, sim, part[1]);
            part[2] = fma((double)p[c].re, sre, part[2]);
            part[2] = fma((double)p[c].im, sim, part[2]);
        }
        FieldIO<FP>::template store<T>(prm.p, prm.vh, prm.nrhs, j, i, p);
        FieldIO<FP>::template store<T>(prm.s, prm.vh, prm.nrhs, j, i, sv);
        FieldIO<HISQ_FP64>::template store<double>(prm.x[j], prm.vh, 1, 0, i, x);
        FieldIO<FP>::template store<T>(prm.r, prm.vh, prm.nrhs, j, i, r);
    }
    vec_block_sum<3, PAIR>(part, lds);
    if (at.leader() && st.go) {
        const size_t o = (size_t)j * gridDim.x + blockIdx.x;
        prm.rr_part[o] = part[0];
        prm.rs_part[o] = part[1];
        prm.ps_part[o] = part[2];
    }
}

// The scalar step and the vector step in one launch, for lattices with few
// partials per column: every block of column j = blockIdx.y sums the
// column's partials (the same values in the same order, so every block takes
// the same decision) and advances its sites.  The state and the <r, r>,
// Re <r, s>, <p, s> partials are double-buffered: state read from st_in and
// written (by block (0, j) alone) to st_out, partials read from set in_buf
// and written to the other, so no block reads what another block of the
// launch writes.  A column waits for its true
// residual while it is inactive with FLAG_CONV or FLAG_RELIABLE; after_check:
// the check block has just formed it.  Block (0, j) also sets the column's
// launch gates: col_off[j] (the iteration's Dslash launches skip the column)
// and tr_skip[j] (the check block skips it).
template <int FP>
__global__ void __launch_bounds__(BLK) cgcg_fused_kernel(CgVecParams prm, const CgScalars *st_in, CgScalars *st_out,
                                                         int *col_off, int after_check, int in_buf) {
    using T = typename Sloppy<FP>::T;
    const int j = blockIdx.y;
    CgScalars s = st_in[j];
    const bool waiting = !s.active && (s.flag == FLAG_CONV || s.flag == FLAG_RELIABLE);
    const bool decide = after_check && waiting;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!s.active && !decide) {
        if (lead)
            st_out[j] = s;
        return;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool site = i < prm.vh;
    // the vectors are loaded before the partial sums so the two overlap
    cplx<T> r[3], w[3], p[3], sv[3];
    cplx<double> x[3];
    if (site) {
        FieldIO<FP>::template load<T>(prm.r, prm.vh, prm.nrhs, j, i, r);
        FieldIO<FP>::template load<T>(prm.w, prm.vh, prm.nrhs, j, i, w);
        FieldIO<FP>::template load<T>(prm.p, prm.vh, prm.nrhs, j, i, p);
        FieldIO<FP>::template load<T>(prm.s, prm.vh, prm.nrhs, j, i, sv);
        FieldIO<HISQ_FP64>::template load<double>(prm.x[j], prm.vh, 1, 0, i, x);
    }
    __shared__ double lds_tot[4];  // apart from lds: a wave may reach block_sum while others still read tot
    __shared__ double lds[12];
    double tot[4];
    cgcg_sums<false>(prm, j, in_buf ? prm.part_buf : 0, tot, lds_tot);
    int wait = -1;
    cgcg_decide(s, tot, decide, &wait);
    if (lead) {
        st_out[j] = s;
        if (wait >= 0)
            prm.tr_skip[j] = wait ? 0 : 1;
        col_off[j] = s.active ? 0 : 1;
    }
    if (!s.go)
        return;
    double part[3] = {0.0, 0.0, 0.0};
    if (site) {
        const bool fresh = s.go == 2;
        const T b = (T)s.beta, a = (T)s.alpha;
        const double ad = s.alpha;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (fresh) {
                p[c] = r[c];
                sv[c] = w[c];
            } else {
                p[c].re = fma(b, p[c].re, r[c].re);
                p[c].im = fma(b, p[c].im, r[c].im);
                sv[c].re = fma(b, sv[c].re, w[c].re);
                sv[c].im = fma(b, sv[c].im, w[c].im);
            }
            x[c].re = fma(ad, (double)p[c].re, x[c].re);
            x[c].im = fma(ad, (double)p[c].im, x[c].im);
            r[c].re = fma(-a, sv[c].re, r[c].re);
            r[c].im = fma(-a, sv[c].im, r[c].im);
            const double rre = r[c].re, rim = r[c].im, sre = sv[c].re, sim = sv[c].im;
            part[0] = fma(rre, rre, part[0]);
            part[0] = fma(rim, rim, part[0]);
            part[1] = fma(rre, sre, part[1]);
            part[1] = fma(rim, sim, part[1]);
            part[2] = fma((double)p[c].re, sre, part[2]);
            part[2] = fma((double)p[c].im, sim, part[2]);
        }
        FieldIO<FP>::template store<T>(prm.p, prm.vh, prm.nrhs, j, i, p);
        FieldIO<FP>::template store<T>(prm.s, prm.vh, prm.nrhs, j, i, sv);
        FieldIO<HISQ_FP64>::template store<double>(prm.x[j], prm.vh, 1, 0, i, x);
        FieldIO<FP>::template store<T>(prm.r, prm.vh, prm.nrhs, j, i, r);
    }
    block_sum<3>(part, lds);
    if (threadIdx.x == 0) {
        const size_t o = (in_buf ? 0 : prm.part_buf) + (size_t)j * gridDim.x + blockIdx.x;
        prm.rr_part[o] = part[0];
        prm.rs_part[o] = part[1];
        prm.ps_part[o] = part[2];
    }
}

// r_j = b_j - ax_j for the ncol columns j of the launch (block row
// blockIdx.y; VecPos) whose tr_skip[j] is 0 (all columns when tr_skip is
// NULL): FP64 inputs b, ax (packed fields of ncol columns), r stored in the
// sloppy precision as column col0 + j of the nf-column field r, block
// partials of ||b_j - ax_j||^2 (FP64 values) in partials[j * gridDim.x +
// block] and, when s and p are not NULL, of Re <r_j, s_j> (the stored r) and
// Re <p_j, s_j> in spart and ppart (same layout; s and p are nf-column fields
// like r).  A launch that forms residuals reopens the iteration launches
// after it: *skip = 0 (nullable) and col_off[j] = 0 (nullable) for each
// column it forms.  PAIR needs col0 even.
template <int FP, bool PAIR>
__global__ void __launch_bounds__(PAIR ? 2 * BLK : BLK)
    residual_cols_kernel(int vh, int ncol, int nf, int col0, const void *b, const void *ax, void *r, double *partials,
                         const int *tr_skip, const void *s, const void *p, double *spart, double *ppart, int *skip,
                         int *col_off) {
    using T = typename Sloppy<FP>::T;
    const VecPos<PAIR> at;
    const int j = at.j;
    const bool run = j < ncol && !(tr_skip && tr_skip[j] != 0);
    if (!PAIR && !run)
        return;  // the whole block belongs to column j
    if (blockIdx.x == 0 && at.leader() && run) {
        if (skip)
            *skip = 0;
        if (col_off)
            col_off[j] = 0;
    }
    __shared__ double lds[vec_lds(3, PAIR)];
    const int i = at.i;
    double part[3] = {0.0, 0.0, 0.0};
    const bool sp = s && p;
    if (run && i < vh) {
        cplx<double> bv[3], av[3];
        FieldIO<HISQ_FP64>::template load<double>(b, vh, ncol, j, i, bv);
        FieldIO<HISQ_FP64>::template load<double>(ax, vh, ncol, j, i, av);
        cplx<T> rv[3], sv[3], pv[3];
        if (sp) {
            FieldIO<FP>::template load<T>(s, vh, nf, col0 + j, i, sv);
            FieldIO<FP>::template load<T>(p, vh, nf, col0 + j, i, pv);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double re = bv[c].re - av[c].re, im = bv[c].im - av[c].im;
            part[0] = fma(re, re, part[0]);
            part[0] = fma(im, im, part[0]);
            rv[c].re = (T)re;
            rv[c].im = (T)im;
            if (sp) {
                part[1] = fma((double)rv[c].re, (double)sv[c].re, part[1]);
                part[1] = fma((double)rv[c].im, (double)sv[c].im, part[1]);
                part[2] = fma((double)pv[c].re, (double)sv[c].re, part[2]);
                part[2] = fma((double)pv[c].im, (double)sv[c].im, part[2]);
            }
        }
        FieldIO<FP>::template store<T>(r, vh, nf, col0 + j, i, rv);
    }
    vec_block_sum<3, PAIR>(part, lds);
    if (at.leader() && run) {
        const size_t o = (size_t)j * gridDim.x + blockIdx.x;
        partials[o] = part[0];
        if (sp) {
            spart[o] = part[1];
            ppart[o] = part[2];
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
        FieldIO<HISQ_FP64>::template load<double>(b, vh, 1, 0, i, bv);
        FieldIO<HISQ_FP64>::template load<double>(ax, vh, 1, 0, i, av);
        cplx<T> rv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double re = bv[c].re - av[c].re, im = bv[c].im - av[c].im;
            part[0] = fma(re, re, part[0]);
            part[0] = fma(im, im, part[0]);
            rv[c].re = (T)re;
            rv[c].im = (T)im;
        }
        FieldIO<FP>::template store<T>(r, vh, 1, 0, i, rv);
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
        FieldIO<HISQ_FP64>::template load<double>(v, vh, 1, 0, i, a);
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
        FieldIO<HISQ_FP64>::template load<double>(a, vh, 1, r, i, u);
        FieldIO<HISQ_FP64>::template load<double>(b, vh, 1, r, i, v);
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
    FieldIO<FS>::template load<T>(src, vh, n, r, i, v);
    FieldIO<FD>::template store<T>(dst, vh, n, r, i, v);
}

// dst (one column) = column k of the n-column field src.
template <int FP>
__global__ void __launch_bounds__(BLK) copy_col_kernel(int vh, int n, int k, const void *src, void *dst) {
    using T = typename Sloppy<FP>::T;
    const int i = blockIdx.x * BLK + threadIdx.x;
    if (i >= vh)
        return;
    cplx<T> v[3];
    FieldIO<FP>::template load<T>(src, vh, n, k, i, v);
    FieldIO<FP>::template store<T>(dst, vh, 1, 0, i, v);
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

// Threads per block of the single-reduction CG vector kernels: 64 on small
// lattices, which 256-thread blocks spread over too few CUs (8^4: 8 blocks
// of 256 against 32 of 64), else 256.  The <r, r> partials of the update
// kernel and of the residual kernel must come from blocks of the same size.
int cg_vec_block(int vh) { return vh <= 32768 ? 64 : BLK; }
int cg_vec_blocks(int vh) { return (vh + cg_vec_block(vh) - 1) / cg_vec_block(vh); }

hipError_t launch_cgcg_step(const CgVecParams &p, int fp, int after_check, hipStream_t st) {
    cgcg_finalize_kernel<<<dim3((unsigned)p.nrhs), 256, 0, st>>>(p, after_check);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int b = cg_vec_block(p.vh);
    const unsigned nb = (unsigned)cg_vec_blocks(p.vh);
    if (fp == HISQ_FP64)
        cgcg_update_kernel<HISQ_FP64, false><<<dim3(nb, (unsigned)p.nrhs), b, 0, st>>>(p);
    else if (p.nrhs >= 2)  // column pairs share 16-byte records
        cgcg_update_kernel<HISQ_FP32, true><<<dim3(nb, (unsigned)(p.nrhs + 1) / 2), 2 * b, 0, st>>>(p);
    else
        cgcg_update_kernel<HISQ_FP32, false><<<dim3(nb, 1u), b, 0, st>>>(p);
    return hipGetLastError();
}

hipError_t launch_residual_cols(int vh, int ncol, int nf, int col0, int fp, const void *b, const void *ax, void *r,
                                double *partials, const int *tr_skip, const void *s, const void *p, double *spart,
                                double *ppart, int *skip, int *col_off, hipStream_t st) {
    const int bs = cg_vec_block(vh);
    const unsigned nb = (unsigned)cg_vec_blocks(vh);
    if (fp == HISQ_FP64)
        residual_cols_kernel<HISQ_FP64, false><<<dim3(nb, (unsigned)ncol), bs, 0, st>>>(
            vh, ncol, nf, col0, b, ax, r, partials, tr_skip, s, p, spart, ppart, skip, col_off);
    else if (ncol >= 2 && col0 % 2 == 0)  // column pairs share 16-byte records
        residual_cols_kernel<HISQ_FP32, true><<<dim3(nb, (unsigned)(ncol + 1) / 2), 2 * bs, 0, st>>>(
            vh, ncol, nf, col0, b, ax, r, partials, tr_skip, s, p, spart, ppart, skip, col_off);
    else
        residual_cols_kernel<HISQ_FP32, false><<<dim3(nb, (unsigned)ncol), bs, 0, st>>>(
            vh, ncol, nf, col0, b, ax, r, partials, tr_skip, s, p, spart, ppart, skip, col_off);
    return hipGetLastError();
}

hipError_t launch_cgcg_fused(const CgVecParams &p, int fp, const CgScalars *st_in, CgScalars *st_out, int *col_off,
                             int after_check, int in_buf, hipStream_t st) {
    const int b = cg_vec_block(p.vh);
    const dim3 g((unsigned)cg_vec_blocks(p.vh), (unsigned)p.nrhs);
    if (fp == HISQ_FP64)
        cgcg_fused_kernel<HISQ_FP64><<<g, b, 0, st>>>(p, st_in, st_out, col_off, after_check, in_buf);
    else
        cgcg_fused_kernel<HISQ_FP32><<<g, b, 0, st>>>(p, st_in, st_out, col_off, after_check, in_buf);
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

hipError_t launch_copy_col(int vh, int fp, int n, int k, const void *src, void *dst, hipStream_t st) {
    if (fp == HISQ_FP64)
        copy_col_kernel<HISQ_FP64><<<grid_for(vh), BLK, 0, st>>>(vh, n, k, src, dst);
    else if (fp == HISQ_FP32)
        copy_col_kernel<HISQ_FP32><<<grid_for(vh), BLK, 0, st>>>(vh, n, k, src, dst);
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
