// PTC network kernels: forward layers, backward (input gradient through the
// adjoint transports, weight gradient as a deterministic reduction over all
// sites), the training loss and Adam.  FP32 fields, FP64 reductions.
#include <algorithm>

#include "dslash.hpp"
#include "internal.hpp"
#include "ptc.hpp"
#include "reduce.hpp"

namespace hisq {

namespace {

constexpr int PB = PTC_BLOCK;

struct Hop {
    int nb;      // half-lattice index of the site read
    int par;     // its parity
    int lblk;    // link parity block
    int lidx;    // link index
    float sg;    // boundary sign
    bool back;   // apply the adjoint
};

// Path p of the layer, at site (par, i): which site and link it reads.
__device__ __forceinline__ Hop path_hop(const Geom &g, const Site &s, int par, int i, int p) {
    Hop h;
    if (p == 0) {
        h.nb = i;
        h.par = par;
        h.lblk = 0;
        h.lidx = 0;
        h.sg = 1.f;
        h.back = false;
        return h;
    }
    const int mu = (p - 1) >> 1;
    const bool fwd = ((p - 1) & 1) == 0;
    const int c = mu == 0 ? s.x : mu == 1 ? s.y : mu == 2 ? s.z : s.t;
    const int n = mu == 0 ? g.nx : mu == 1 ? g.ny : mu == 2 ? g.nz : g.nt;
    const int stride = mu == 1 ? g.hx : mu == 2 ? g.hx * g.ny : g.hx * g.ny * g.nz;
    neighbour<float>(g, i, c, n, stride, mu, fwd ? +1 : -1, h.nb, h.sg);
    h.par = 1 - par;
    h.lblk = fwd ? par : 1 - par;
    h.lidx = fwd ? i : h.nb;
    h.back = !fwd;
    return h;
}

__device__ __forceinline__ void transport(const float m[18], bool back, float sg, const cplx<float> v[3],
                                          cplx<float> t[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        t[a].re = t[a].im = 0.f;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (!back)
                cmac(t[a], m[6 * a + 2 * b], m[6 * a + 2 * b + 1], v[b]);
            else
                cmac_conj(t[a], m[6 * b + 2 * a], m[6 * b + 2 * a + 1], v[b]);
        }
        t[a].re *= sg;
        t[a].im *= sg;
    }
}

__device__ __forceinline__ const char *xblock(const char *links, int par, int mu, int vh) {
    return links + link_block<HISQ_FP32>(0, par, mu, vh);
}

// out_co(x) = sum_ci sum_p w[co][ci][p] (T_p in_ci)(x), one thread per site.
// IN_EVEN: the input is zero on the odd sites (the first layer), so the paths
// that read odd sites are left out (an even site keeps the identity path, an
// odd site the eight hops).  OUT_EVEN: only the even output sites are formed
// (the last layer, whose odd sites nothing reads).  The launch does nothing
// while skip (nullable) points to a nonzero value.
template <int CIN, int COUT, bool IN_EVEN, bool OUT_EVEN>
__global__ void __launch_bounds__(PB) layer_fwd_kernel(Geom g, const char *links, const float2 *w, const void *in,
                                                       void *out, const int *skip) {
    if (skip && *skip)
        return;
    const int gid = blockIdx.x * PB + threadIdx.x;
    if (gid >= (OUT_EVEN ? 1 : 2) * g.vh)
        return;
    const int par = gid >= g.vh;
    const int i = gid - par * g.vh;
    const Site s = site_coords(g, par, i);
    cplx<float> acc[COUT][3];
#pragma unroll
    for (int co = 0; co < COUT; ++co)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            acc[co][a].re = acc[co][a].im = 0.f;
#pragma unroll
    for (int p = 0; p < PTC_PATHS; ++p) {
        const Hop h = path_hop(g, s, par, i, p);
        if (IN_EVEN && h.par == 1)
            continue;
        float m[18];
        if (p > 0)
            LinkIO<HISQ_FP32>::load(xblock(links, h.lblk, (p - 1) >> 1, g.vh), g.vh, h.lidx, m);
        for (int ci = 0; ci < CIN; ++ci) {
            cplx<float> v[3], t[3];
            FieldIO<HISQ_FP32>::template load<float>(in, g.vh, 1, 2 * ci + h.par, h.nb, v);
            if (p > 0) {
                transport(m, h.back, h.sg, v, t);
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    t[a] = v[a];
            }
#pragma unroll
            for (int co = 0; co < COUT; ++co) {
                const float2 wv = w[(co * CIN + ci) * PTC_PATHS + p];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    cmac(acc[co][a], wv.x, wv.y, t[a]);
            }
        }
    }
#pragma unroll
    for (int co = 0; co < COUT; ++co)
        FieldIO<HISQ_FP32>::template store<float>(out, g.vh, 1, 2 * co + par, i, acc[co]);
}

// g_in_ci(x) = sum_p T_p^+ (sum_co conj(w[co][ci][p]) g_co)(x); T_{+mu}^+ = T_{-mu}.
// GOUT_EVEN: g_out is zero on the odd sites (the last layer), so the paths
// that read odd sites are left out; OUT_EVEN: only the even sites of g_in are
// formed (the first layer, whose input gradient is read on the even sites).
template <int CIN, int COUT, bool GOUT_EVEN, bool OUT_EVEN>
__global__ void __launch_bounds__(PB) layer_bwd_in_kernel(Geom g, const char *links, const float2 *w,
                                                          const void *gout, void *gin) {
    const int gid = blockIdx.x * PB + threadIdx.x;
    if (gid >= (OUT_EVEN ? 1 : 2) * g.vh)
        return;
    const int par = gid >= g.vh;
    const int i = gid - par * g.vh;
    const Site s = site_coords(g, par, i);
    cplx<float> acc[CIN][3];
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            acc[ci][a].re = acc[ci][a].im = 0.f;
#pragma unroll
    for (int p = 0; p < PTC_PATHS; ++p) {
        // adjoint of path p is the opposite hop
        const int padj = p == 0 ? 0 : (((p - 1) & 1) == 0 ? p + 1 : p - 1);
        const Hop h = path_hop(g, s, par, i, padj);
        if (GOUT_EVEN && h.par == 1)
            continue;
        float m[18];
        if (p > 0)
            LinkIO<HISQ_FP32>::load(xblock(links, h.lblk, (p - 1) >> 1, g.vh), g.vh, h.lidx, m);
        for (int co = 0; co < COUT; ++co) {
            cplx<float> v[3], t[3];
            FieldIO<HISQ_FP32>::template load<float>(gout, g.vh, 1, 2 * co + h.par, h.nb, v);
            if (p > 0) {
                transport(m, h.back, h.sg, v, t);
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    t[a] = v[a];
            }
#pragma unroll
            for (int ci = 0; ci < CIN; ++ci) {
                const float2 wv = w[(co * CIN + ci) * PTC_PATHS + p];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    cmac_conj(acc[ci][a], wv.x, wv.y, t[a]);
            }
        }
    }
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci)
        FieldIO<HISQ_FP32>::template store<float>(gin, g.vh, 1, 2 * ci + par, i, acc[ci]);
}

// Block partials of dL/dw[co][ci][p] = sum_x <(T_p in_ci)(x), g_co(x)>, one
// thread per site for all (ci, p) pairs: g_out of the site and each path's
// link are loaded once and reused by every input channel.  Each wave sums
// its 2 COUT values of a pair (halving exchanges, in FP32: 64 products of
// FP32 values) into LDS as FP64 without a block barrier; at the end the block
// adds the waves in order (deterministic, FP64) into
// partials[(pair * 2 COUT + k) * gridDim.x + blockIdx.x], pair = ci * 9 + p.
// IN_EVEN: the input is zero on odd sites (paths reading them contribute 0);
// GOUT_EVEN: g_out is zero on odd sites, so only the even sites are summed.
template <int CIN, int COUT, bool IN_EVEN, bool GOUT_EVEN>
__global__ void __launch_bounds__(PB) layer_bwd_w_kernel(Geom g, const char *links, const void *in,
                                                         const void *gout, double *partials) {
    constexpr int NV = 2 * COUT;
    constexpr int NPAIR = CIN * PTC_PATHS;
    __shared__ double lds[(PB / 64) * NPAIR * NV];  // per wave, per pair, NV totals
    const int gid = blockIdx.x * PB + threadIdx.x;
    const bool valid = gid < (GOUT_EVEN ? 1 : 2) * g.vh;
    const int par = valid && gid >= g.vh;
    const int i = valid ? gid - par * g.vh : 0;
    const Site s = site_coords(g, par, i);
    cplx<float> gv[COUT][3];
#pragma unroll
    for (int co = 0; co < COUT; ++co) {
        if (valid) {
            FieldIO<HISQ_FP32>::template load<float>(gout, g.vh, 1, 2 * co + par, i, gv[co]);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                gv[co][a].re = gv[co][a].im = 0.f;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int p = 0; p < PTC_PATHS; ++p) {
        const Hop h = path_hop(g, s, par, i, p);
        const bool use = valid && !(IN_EVEN && h.par == 1);
        float m[18];
        if (p > 0 && use)
            LinkIO<HISQ_FP32>::load(xblock(links, h.lblk, (p - 1) >> 1, g.vh), g.vh, h.lidx, m);
        for (int ci = 0; ci < CIN; ++ci) {
            float acc[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k)
                acc[k] = 0.f;
            if (use) {
                cplx<float> v[3], t[3];
                FieldIO<HISQ_FP32>::template load<float>(in, g.vh, 1, 2 * ci + h.par, h.nb, v);
                if (p > 0) {
                    transport(m, h.back, h.sg, v, t);
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        t[a] = v[a];
                }
#pragma unroll
                for (int co = 0; co < COUT; ++co) {
                    // conj(t) . g over the colours in FP32, widened once per value
                    float re = 0.f, im = 0.f;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        re = fmaf(t[a].re, gv[co][a].re, fmaf(t[a].im, gv[co][a].im, re));
                        im = fmaf(t[a].re, gv[co][a].im, fmaf(-t[a].im, gv[co][a].re, im));
                    }
                    acc[2 * co] = re;
                    acc[2 * co + 1] = im;
                }
            }
            wave_sum_multi<NV>(acc);
            if ((lane & (64 / NV - 1)) == 0)
                lds[(wave * NPAIR + ci * PTC_PATHS + p) * NV + wave_multi_index<NV>(lane)] = (double)acc[0];
        }
    }
    // one barrier per block: the waves' totals of every pair, added in wave order
    __syncthreads();
    for (int k = threadIdx.x; k < NPAIR * NV; k += PB) {
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < PB / 64; ++w)
            tot += lds[w * NPAIR * NV + k];
        partials[(size_t)k * gridDim.x + blockIdx.x] = tot;
    }
}

// Weight gradient of the 8 -> 8 layer as a contraction over the sites,
//   G[co][ci][p] = sum_x sum_a conj((T_p in_ci)(x)_a) gout_co(x)_a,
// in tiles of WG_S sites (both parities).  Phase 1: thread t forms, for tile
// site s = t % WG_S and input channel ci = t / WG_S, the nine transported
// vectors of ci, and the output gradient of channel ci at s, into LDS.
// Phase 2: thread t accumulates the outputs co = t % 8, q = ci * 9 + p in
// {t / 8, t / 8 + 32, t / 8 + 64 (< 72)} over the tile's sites and colours in
// FP32 (the per-site products are FP32) and adds the tile's sums to FP64
// totals.  The block walks the tiles with stride gridDim.x and writes its
// totals as the block partials of layer_bwd_w_kernel's layout (summed by
// wgrad_reduce_kernel).  No sum runs across a wavefront per site and
// (channel, path) pair, as in layer_bwd_w_kernel: 8 -> 8 layer at 32^4
// 1.89 -> 1.04 ms.
constexpr int WG_S = 32;

__global__ void __launch_bounds__(256) wgrad88_kernel(Geom g, const char *links, const void *in, const void *gout,
                                                      double *partials) {
    constexpr int NQ = PTC_CH * PTC_PATHS;  // 72 (channel, path) pairs
    __shared__ float2 ts[WG_S][NQ][3];
    __shared__ float2 gs[WG_S][PTC_CH][3];
    const int nsites = 2 * g.vh;
    const int ntiles = (nsites + WG_S - 1) / WG_S;
    const int t = threadIdx.x;
    const int co = t & 7, qb = t >> 3;
    double tot[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        {
            const int sl = t % WG_S, ci = t / WG_S;
            const int gid = tile * WG_S + sl;
            const bool valid = gid < nsites;
            const int par = valid && gid >= g.vh;
            const int i = valid ? gid - par * g.vh : 0;
            const Site st = site_coords(g, par, i);
            cplx<float> gv[3];
            if (valid) {
                FieldIO<HISQ_FP32>::template load<float>(gout, g.vh, 1, 2 * ci + par, i, gv);
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    gv[a].re = gv[a].im = 0.f;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
                gs[sl][ci][a] = make_float2(gv[a].re, gv[a].im);
#pragma unroll
            for (int p = 0; p < PTC_PATHS; ++p) {
                cplx<float> tv[3];
                if (valid) {
                    const Hop h = path_hop(g, st, par, i, p);
                    cplx<float> v[3];
                    FieldIO<HISQ_FP32>::template load<float>(in, g.vh, 1, 2 * ci + h.par, h.nb, v);
                    if (p > 0) {
                        float m[18];
                        LinkIO<HISQ_FP32>::load(xblock(links, h.lblk, (p - 1) >> 1, g.vh), g.vh, h.lidx, m);
                        transport(m, h.back, h.sg, v, tv);
                    } else {
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            tv[a] = v[a];
                    }
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        tv[a].re = tv[a].im = 0.f;
                }
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    ts[sl][ci * PTC_PATHS + p][a] = make_float2(tv[a].re, tv[a].im);
            }
        }
        __syncthreads();
        float acc[3][2] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
        const bool third = qb + 64 < NQ;  // uniform over the wavefront
        for (int sl = 0; sl < WG_S; ++sl) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float2 gg = gs[sl][co][a];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    if (k < 2 || third) {
                        const float2 tt = ts[sl][qb + 32 * k][a];
                        acc[k][0] = fmaf(tt.x, gg.x, fmaf(tt.y, gg.y, acc[k][0]));
                        acc[k][1] = fmaf(tt.x, gg.y, fmaf(-tt.y, gg.x, acc[k][1]));
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            tot[k][0] += (double)acc[k][0];
            tot[k][1] += (double)acc[k][1];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int q = qb + 32 * k;
        if (q < NQ) {
            const size_t slot = (size_t)q * 2 * PTC_CH + 2 * co;  // pair q, output channel co, re / im
            partials[slot * gridDim.x + blockIdx.x] = tot[k][0];
            partials[(slot + 1) * gridDim.x + blockIdx.x] = tot[k][1];
        }
    }
}

// grad[(co * CIN + ci) * 9 + p] += sum over the nblk block partials, one
// wavefront per real value (slot = pair * 2 COUT + 2 co + re/im), summed in a
// fixed order (wave_sum_slot).
__global__ void __launch_bounds__(256) wgrad_reduce_kernel(int cin, int cout, int nblk, const double *partials,
                                                           double2 *grad) {
    const int slot = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int nslots = cin * PTC_PATHS * cout * 2;
    if (slot >= nslots)  // uniform over the wavefront
        return;
    const double sum = wave_sum_slot(partials + (size_t)slot * nblk, nblk);
    if ((threadIdx.x & 63) != 0)
        return;
    const int pair = slot / (2 * cout);
    const int rem = slot - pair * 2 * cout;
    const int co = rem >> 1, part = rem & 1;
    const int ci = pair / PTC_PATHS, p = pair - ci * PTC_PATHS;
    double2 *dst = grad + (co * cin + ci) * PTC_PATHS + p;
    if (part == 0)
        dst->x += sum;
    else
        dst->y += sum;
}

// a0 = (in_even, 0 on odd sites), channel 0.
__global__ void embed_kernel(int vh, const void *in_even, void *a0, const int *skip) {
    if (skip && *skip)
        return;
    const int gid = blockIdx.x * PB + threadIdx.x;
    if (gid >= 2 * vh)
        return;
    const int par = gid >= vh;
    const int i = gid - par * vh;
    cplx<float> v[3];
    if (par == 0) {
        FieldIO<HISQ_FP32>::template load<float>(in_even, vh, 1, 0, i, v);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            v[a].re = v[a].im = 0.f;
    }
    FieldIO<HISQ_FP32>::template store<float>(a0, vh, 1, par, i, v);
}

__global__ void extract_kernel(int vh, const void *a3, void *out_even, const int *skip) {
    if (skip && *skip)
        return;
    const int i = blockIdx.x * PB + threadIdx.x;
    if (i >= vh)
        return;
    cplx<float> v[3];
    FieldIO<HISQ_FP32>::template load<float>(a3, vh, 1, 0, i, v);
    FieldIO<HISQ_FP32>::template store<float>(out_even, vh, 1, 0, i, v);
}

// Block partials of Re <x, b> for the FP64 solution x and FP32 source b
// (even sites).
__global__ void __launch_bounds__(PB) xb_kernel(int vh, const void *x64, const void *b32, double *partials) {
    __shared__ double lds[4];
    const int i = blockIdx.x * PB + threadIdx.x;
    double part[1] = {0.0};
    if (i < vh) {
        cplx<double> x[3];
        cplx<float> b[3];
        FieldIO<HISQ_FP64>::template load<double>(x64, vh, 1, 0, i, x);
        FieldIO<HISQ_FP32>::template load<float>(b32, vh, 1, 0, i, b);
#pragma unroll
        for (int a = 0; a < 3; ++a)
            part[0] += x[a].re * (double)b[a].re + x[a].im * (double)b[a].im;
    }
    block_sum<1>(part, lds);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = part[0];
}

// e = y - x on even sites (y: network output, channel 0 of a3; x: FP64).
__global__ void __launch_bounds__(PB) diff_kernel(int vh, const void *a3, const void *x64, void *e) {
    const int i = blockIdx.x * PB + threadIdx.x;
    if (i >= vh)
        return;
    cplx<float> y[3], d[3];
    cplx<double> x[3];
    FieldIO<HISQ_FP32>::template load<float>(a3, vh, 1, 0, i, y);
    FieldIO<HISQ_FP64>::template load<double>(x64, vh, 1, 0, i, x);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d[a].re = (float)((double)y[a].re - x[a].re);
        d[a].im = (float)((double)y[a].im - x[a].im);
    }
    FieldIO<HISQ_FP32>::template store<float>(e, vh, 1, 0, i, d);
}

// Output gradient of L_i = <e, A e> / c (c = <x, b>), scaled by 1/B:
// g3 = 2 A e / (B c) on even sites, 0 on odd sites; *loss_acc += <e, A e> / (B c).
__global__ void __launch_bounds__(PB) energy_grad_kernel(int vh, const void *Ae, const double *eAe,
                                                         const double *c, double inv_batch, void *g3,
                                                         double *loss_acc) {
    const int gid = blockIdx.x * PB + threadIdx.x;
    const double cc = *c;
    if (gid == 0)
        *loss_acc += *eAe * inv_batch / cc;
    if (gid >= 2 * vh)
        return;
    const int par = gid >= vh;
    const int i = gid - par * vh;
    cplx<float> gv[3];
    if (par == 0) {
        cplx<float> v[3];
        FieldIO<HISQ_FP32>::template load<float>(Ae, vh, 1, 0, i, v);
        const float coef = (float)(2.0 * inv_batch / cc);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            gv[a].re = coef * v[a].re;
            gv[a].im = coef * v[a].im;
        }
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            gv[a].re = gv[a].im = 0.f;
    }
    FieldIO<HISQ_FP32>::template store<float>(g3, vh, 1, par, i, gv);
}

// Adam on real and imaginary parts as separate parameters; FP64 master
// weights and moments, FP32 copy for the kernels.
__global__ void adam_kernel(double2 *w, float2 *w32, const double2 *g, double2 *m, double2 *v, int step, double lr,
                            double b1, double b2, double eps) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= PTC_NW)
        return;
    const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    double2 wk = w[k], gk = g[k], mk = m[k], vk = v[k];
    mk.x = b1 * mk.x + (1.0 - b1) * gk.x;
    mk.y = b1 * mk.y + (1.0 - b1) * gk.y;
    vk.x = b2 * vk.x + (1.0 - b2) * gk.x * gk.x;
    vk.y = b2 * vk.y + (1.0 - b2) * gk.y * gk.y;
    wk.x -= lr * (mk.x / c1) / (sqrt(vk.x / c2) + eps);
    wk.y -= lr * (mk.y / c1) / (sqrt(vk.y / c2) + eps);
    w[k] = wk;
    m[k] = mk;
    v[k] = vk;
    w32[k] = make_float2((float)wk.x, (float)wk.y);
}

__global__ void fill_f64_kernel(double *p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0.0;
}

inline unsigned nb(int64_t n) { return (unsigned)((n + PB - 1) / PB); }

}  // namespace

int ptc_blocks(const Geom &g) { return (int)nb(2 * (int64_t)g.vh); }

hipError_t ptc_embed(const Geom &g, const void *in_even, void *a0, hipStream_t st, const int *skip) {
    embed_kernel<<<nb(2 * (int64_t)g.vh), PB, 0, st>>>(g.vh, in_even, a0, skip);
    return hipGetLastError();
}

hipError_t ptc_extract(const Geom &g, const void *a3, void *out_even, hipStream_t st, const int *skip) {
    extract_kernel<<<nb(g.vh), PB, 0, st>>>(g.vh, a3, out_even, skip);
    return hipGetLastError();
}

// The three layers of the 1 -> 8 -> 8 -> 1 network: layer 1 reads an input
// that is zero on odd sites, layer 3's output is read on even sites only.
hipError_t ptc_layer_fwd(const Geom &g, int cin, int cout, const char *links, const float2 *w, const void *in,
                         void *out, hipStream_t st, const int *skip) {
    const dim3 full(nb(2 * (int64_t)g.vh)), even(nb(g.vh));
    if (cin == 1 && cout == PTC_CH)
        layer_fwd_kernel<1, PTC_CH, true, false><<<full, PB, 0, st>>>(g, links, w, in, out, skip);
    else if (cin == PTC_CH && cout == PTC_CH)
        layer_fwd_kernel<PTC_CH, PTC_CH, false, false><<<full, PB, 0, st>>>(g, links, w, in, out, skip);
    else if (cin == PTC_CH && cout == 1)
        layer_fwd_kernel<PTC_CH, 1, false, true><<<even, PB, 0, st>>>(g, links, w, in, out, skip);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Backward through the same layers: layer 3's output gradient is zero on odd
// sites, layer 1's input gradient is needed on even sites only.
hipError_t ptc_layer_bwd_in(const Geom &g, int cin, int cout, const char *links, const float2 *w,
                            const void *g_out, void *g_in, hipStream_t st) {
    const dim3 full(nb(2 * (int64_t)g.vh)), even(nb(g.vh));
    if (cin == PTC_CH && cout == PTC_CH)
        layer_bwd_in_kernel<PTC_CH, PTC_CH, false, false><<<full, PB, 0, st>>>(g, links, w, g_out, g_in);
    else if (cin == PTC_CH && cout == 1)
        layer_bwd_in_kernel<PTC_CH, 1, true, false><<<full, PB, 0, st>>>(g, links, w, g_out, g_in);
    else if (cin == 1 && cout == PTC_CH)
        layer_bwd_in_kernel<1, PTC_CH, false, true><<<even, PB, 0, st>>>(g, links, w, g_out, g_in);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t ptc_layer_bwd_w(const Geom &g, int cin, int cout, const char *links, const void *in, const void *g_out,
                           double *partials, double2 *grad, hipStream_t st) {
    int nblk = ptc_blocks(g);
    if (cin == 1 && cout == PTC_CH)
        layer_bwd_w_kernel<1, PTC_CH, true, false><<<dim3((unsigned)nblk), PB, 0, st>>>(g, links, in, g_out, partials);
    else if (cin == PTC_CH && cout == PTC_CH) {
        nblk = std::min(nblk, 1024);  // blocks walk the tiles; the partials hold ptc_blocks(g) per slot
        wgrad88_kernel<<<dim3((unsigned)nblk), 256, 0, st>>>(g, links, in, g_out, partials);
    }
    else if (cin == PTC_CH && cout == 1) {
        nblk = nb(g.vh);  // the even sites only
        layer_bwd_w_kernel<PTC_CH, 1, false, true><<<dim3((unsigned)nblk), PB, 0, st>>>(g, links, in, g_out, partials);
    } else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int nslots = cin * PTC_PATHS * cout * 2;
    wgrad_reduce_kernel<<<(nslots + 3) / 4, 256, 0, st>>>(cin, cout, nblk, partials, grad);
    return hipGetLastError();
}

hipError_t ptc_xb(const Geom &g, const void *x64, const void *b32, double *partials, double *out, hipStream_t st) {
    xb_kernel<<<nb(g.vh), PB, 0, st>>>(g.vh, x64, b32, partials);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? launch_sum_partials(partials, 1, nb(g.vh), out, 1, nullptr, st) : e;
}

hipError_t ptc_diff(const Geom &g, const void *a3, const void *x64, void *e, hipStream_t st) {
    diff_kernel<<<nb(g.vh), PB, 0, st>>>(g.vh, a3, x64, e);
    return hipGetLastError();
}

hipError_t ptc_energy_grad(const Geom &g, const void *Ae, const double *eAe, const double *c, double inv_batch,
                           void *g3, double *loss_acc, hipStream_t st) {
    energy_grad_kernel<<<nb(2 * (int64_t)g.vh), PB, 0, st>>>(g.vh, Ae, eAe, c, inv_batch, g3, loss_acc);
    return hipGetLastError();
}

hipError_t ptc_adam(double2 *w_master, float2 *w_f32, const double2 *grad, double2 *m, double2 *v, int step,
                    double lr, double b1, double b2, double eps, hipStream_t st) {
    adam_kernel<<<(PTC_NW + 255) / 256, 256, 0, st>>>(w_master, w_f32, grad, m, v, step, lr, b1, b2, eps);
    return hipGetLastError();
}

hipError_t ptc_fill_f64(double *p, size_t n, hipStream_t st) {
    if (n == 0)
        return hipSuccess;
    fill_f64_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n);
    return hipGetLastError();
}

}  // namespace hisq
