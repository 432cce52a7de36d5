// The even/odd HISQ Dslash on gfx950.
//
// Two thread mappings, chosen per problem by the autotuner:
//  * SITE:  one thread per output site; NIN right-hand sides per thread share
//           every link load (the N_inner loop of the paper's Sec. 5.1); the
//           N_outer groups of NIN right-hand sides are further blocks.
//  * DIR:   four consecutive lanes per output site, lane mu handling the four
//           hops (+-1, +-3) along direction mu; the partial sums are combined
//           by two butterfly shuffles.  Four times the wavefronts of SITE, so
//           a 32^3x8 lattice fills all 256 CUs with more loads in flight.
// Both read every link matrix exactly once per application, as 16-byte
// coalesced chunks of the structure-of-arrays link layout.  The right-hand
// side group is the fastest-varying part of the block index, so the N_outer
// blocks of one range of sites run together (on one XCD when remapped) and
// its links come from cache after the first of them.
#pragma once

#include "access.hpp"
#include "reduce.hpp"

namespace hisq {

enum { VAR_SITE = 0, VAR_DIR = 1, VAR_LDS = 2, VAR_HOP = 3 };
// EPI_PLAIN: out = D in.  EPI_AXPY: out = ad * D in + ay * y.
// EPI_AXPY_DOT: as EPI_AXPY, and dot_out[r] = Re <y_r, out_r> (FP64 sums,
// deterministic: block partials summed in block order by the last block).
enum { EPI_PLAIN = 0, EPI_AXPY = 1, EPI_AXPY_DOT = 2 };

struct DslashParams {
    Geom g;
    int out_parity;
    int nrhs;
    int xcd_remap;  // map consecutive workgroups of one XCD to neighbouring sites
    int band;       // y-rows per band in the z-slab block order
    const char *links;
    const void *in;
    void *out;
    const void *y;  // EPI_AXPY*: out = ad * D in + ay * y (y on the output parity)
    double ad, ay;
    int ay_per_rhs;                 // EPI_AXPY*: use ay_rhs[r] instead of ay
    double ay_rhs[HISQ_MAX_RHS];
    const int *skip;     // optional: if *skip != 0 the whole launch does nothing
    // optional [nrhs]: a block whose right-hand sides r all have
    // col_skip[r] != 0 does nothing (its outputs and partials are not written)
    const int *col_skip;
    double *partials;    // EPI_AXPY_DOT: [nrhs][site blocks] block partials
    double *dot_out;     // EPI_AXPY_DOT: totals, dot_out[r * dot_stride] (finalize kernel)
    int dot_stride;
};

// Coordinates of half-lattice site i of parity p.
struct Site {
    int x, y, z, t;
};

__device__ __forceinline__ Site site_coords(const Geom &g, int p, int i) {
    Site s;
    const int xh = i % g.hx;
    int rest = i / g.hx;
    s.y = rest % g.ny;
    rest /= g.ny;
    s.z = rest % g.nz;
    s.t = rest / g.nz;
    s.x = 2 * xh + ((s.y + s.z + s.t + p) & 1);
    return s;
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip.  With
// remapping (block order 1 or 2), XCD k works on one contiguous range of
// logical blocks (nearby sites), so neighbour colour vectors are shared within
// that XCD's L2.
__device__ __forceinline__ int logical_block(int remap) {
    const int b = blockIdx.x;
    if (!remap)
        return b;
    const int G = gridDim.x;
    const int q = G >> 3, r = G & 7;
    const int x = b & 7, j = b >> 3;
    return x * q + min(x, r) + j;
}

// Block coordinates: site block `sb` (of nsb) and first right-hand side r0
// of the block's group of NIN.
// Traversal position ip -> site index when the XCDs take z-slabs (block
// order 2): ip runs over (slab, y-band, t, z within the slab, y within the
// band, x/2) with 8 slabs of N_z / 8 planes, so the contiguous range of XCD k
// is slab k for every t; its hops in t stay inside the slab and only the
// +-1/+-3 hops in z reach other XCDs' sites.  Cutting the slab into bands of
// `band` y-rows (band divides N_y; band = N_y: no cut) shortens the distance
// between the first and the last use of a vector by the t-hops, which matters
// once several right-hand sides make each site's vectors large.  Requires N_z
// divisible by 8.
__device__ __forceinline__ int zslab_site(const Geom &g, int ip, int band) {
    const int piece = band * g.hx;  // sites of one (t, z, band) piece of this parity
    const int zw = g.nz >> 3;
    const int q = ip / piece, r = ip - q * piece;
    const int zl = q % zw;
    int st = q / zw;
    const int t = st % g.nt;
    st /= g.nt;
    const int nb = g.ny / band;
    const int bd = st % nb, slab = st / nb;
    return (t * g.nz + slab * zw + zl) * (g.ny * g.hx) + bd * piece + r;
}

// y-rows per band of the z-slab order: whole planes for one right-hand side
// (32^3x8: unbanded is fastest), bands of 8 rows for several (16 rhs at
// 48^3x12: FP64 1231 -> 1105 us, FP32 600 -> 585 us).
inline int zslab_band(const Geom &g, int nrhs) { return nrhs > 1 && g.ny % 8 == 0 ? 8 : g.ny; }

template <int NIN> struct BlockPos {
    int sb, nsb, r0, nr;
    // site index of traversal position ip (ip < vh)
    __device__ __forceinline__ int site(const DslashParams &prm, int ip) const {
        return prm.xcd_remap == 2 && ip < prm.g.vh ? zslab_site(prm.g, ip, prm.band) : ip;
    }
    __device__ __forceinline__ BlockPos(const DslashParams &prm) {
        const int nouter = (prm.nrhs + NIN - 1) / NIN;
        const int lb = logical_block(prm.xcd_remap);
        sb = lb / nouter;
        nsb = gridDim.x / nouter;
        r0 = (lb - sb * nouter) * NIN;
        nr = min(NIN, prm.nrhs - r0);
    }
};

// False when col_skip gates off every right-hand side of this block.
template <int NIN> __device__ __forceinline__ bool columns_run(const DslashParams &prm, const BlockPos<NIN> &bp) {
    if (!prm.col_skip)
        return true;
    int run = 0;
    for (int r = 0; r < bp.nr; ++r)
        run |= prm.col_skip[bp.r0 + r] == 0 ? 1 : 0;
    return run != 0;
}

template <int NIN, typename A> __device__ __forceinline__ void zero(cplx<A> (&v)[NIN][3]) {
#pragma unroll
    for (int r = 0; r < NIN; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            v[r][a].re = v[r][a].im = (A)0;
}

// Half-lattice index and time-boundary sign of the neighbour `step` sites
// along mu of a site with coordinate c (extent n, half-index stride `stride`).
template <typename A>
__device__ __forceinline__ void neighbour(const Geom &g, int i, int c, int n, int stride, int mu, int step,
                                          int &nb, A &sg) {
    int v = c + step;
    const bool wrap = v >= n || v < 0;
    v = v >= n ? v - n : (v < 0 ? v + n : v);
    nb = mu == 0 ? i + ((v >> 1) - (c >> 1)) : i + (v - c) * stride;
    sg = (wrap && mu == 3) ? (A)g.t_bc : (A)1;
}

// Registers of one hop: the link and the NIN neighbour vectors.
template <int NIN, typename A> struct HopBuf {
    A m[18];
    cplx<A> v[NIN][3];
};

// Whether column r (< NIN, unrolled) of a group of nr >= 1 columns is there.
// ONE: the caller knows that the group is one column, and the test folds away,
// which keeps the loads and their use out of a branch.  A field load in a
// branch of its own had its binary16 conversion placed beside it in that
// branch, so every hop of the FP16N one-column kernel waited for all of the
// next hop's loads before computing the current one (32^3x8 FP16N 14.5 ->
// 13.9 us, FP64 47.9 -> 46.8 us).  The one-column site kernel takes it with
// every epilogue (FP64 CG 16.9 -> 16.6 ms; before eta was folded into the hop
// signs the FP64 kernel with the fused dot product ran 46 -> 53 us with it);
// with several columns the compiler hoisted more loads than the register file
// holds.
template <bool ONE> __device__ __forceinline__ constexpr bool has_col(int r, int nr) { return ONE || r < nr; }

// tmp += U v (or -U^+ v) with v = sg * (neighbour vectors in b); row 2 of a
// compressed link (field f) is rebuilt here, after its loads have landed.
template <int LP, int NIN, typename A, bool ONE = false>
__device__ __forceinline__ void hop_apply(const HopBuf<NIN, A> &bin, bool back, A sg, int nr,
                                          cplx<A> (&tmp)[NIN][3], int f) {
    HopBuf<NIN, A> b = bin;
    if constexpr (LinkIO<LP>::rebuild)
        LinkIO<LP>::finish(b.m, f);
#pragma unroll
    for (int r = 0; r < NIN; ++r) {
        if (has_col<ONE>(r, nr)) {
            cplx<A> v[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[c].re = b.v[r][c].re * sg;
                v[c].im = b.v[r][c].im * sg;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (!back)
                        cmac(tmp[r][a], b.m[6 * a + 2 * c], b.m[6 * a + 2 * c + 1], v[c]);
                    else  // -(U^+)_{ac} v_c = -conj(U_{ca}) v_c
                        cmac_conj(tmp[r][a], -b.m[6 * c + 2 * a], -b.m[6 * c + 2 * a + 1], v[c]);
                }
        }
    }
}

template <int LP, int FP, int NIN, typename A, bool NT>
__device__ __forceinline__ void hop_load(HopBuf<NIN, A> &b, const char *blk, int vh, int ilink, const void *in,
                                         int ipsi, int ncol, int r0, int nr, int f) {
    LinkIO<LP>::template load<NT>(blk, vh, ilink, b.m, f);
    load_group<FP, NIN, A>(in, vh, ncol, r0, nr, ipsi, b.v);
}

// The nr (<= NIN) columns r0 .. r0 + nr - 1 of site i of an ncol-column
// field.  FP32 fields with NIN even take both slots of each pair with one
// 16-byte access per colour (r0 is a multiple of NIN, so the group starts on
// a pair; the pair of an odd last column has an unused second slot, which
// is loaded and never used, and stored as zero).
template <int FP, int NIN, typename A, bool ONE = false>
__device__ __forceinline__ void load_group(const void *f, int vh, int ncol, int r0, int nr, int i,
                                           cplx<A> (&v)[NIN][3]) {
    if constexpr (FP == HISQ_FP32 && NIN % 2 == 0) {
#pragma unroll
        for (int r = 0; r < NIN; r += 2)
            if (has_col<ONE>(r, nr))
                FieldIO<FP>::template load_pair<A>(f, vh, (r0 + r) >> 1, i, v[r], v[r + 1]);
    } else {
#pragma unroll
        for (int r = 0; r < NIN; ++r)
            if (has_col<ONE>(r, nr))
                FieldIO<FP>::template load<A>(f, vh, ncol, r0 + r, i, v[r]);
    }
}

template <int FP, int NIN, typename A, bool ONE = false>
__device__ __forceinline__ void store_group(void *f, int vh, int ncol, int r0, int nr, int i,
                                            const cplx<A> (&v)[NIN][3]) {
    if constexpr (FP == HISQ_FP32 && NIN % 2 == 0) {
#pragma unroll
        for (int r = 0; r < NIN; r += 2)
            if (has_col<ONE>(r, nr))
                FieldIO<FP>::template store_pair<A>(f, vh, (r0 + r) >> 1, i, v[r], v[r + 1]);
    } else {
#pragma unroll
        for (int r = 0; r < NIN; ++r)
            if (has_col<ONE>(r, nr))
                FieldIO<FP>::template store<A>(f, vh, ncol, r0 + r, i, v[r]);
    }
}

// The four hops along direction mu (runtime) of site s (half index i, parity
// p), times eta_mu(s), accumulated into acc.  The loads of the next hop are
// issued before the current hop is computed.
template <int LP, int FP, int NIN, typename A, bool NT>
__device__ __forceinline__ void dslash_direction(const Geom &g, int p, const char *links, const void *in,
                                                 int i, const Site &s, int mu, int ncol, int r0, int nr,
                                                 cplx<A> (&acc)[NIN][3]) {
    const int vh = g.vh;
    const int c = mu == 0 ? s.x : mu == 1 ? s.y : mu == 2 ? s.z : s.t;
    const int n = mu == 0 ? g.nx : mu == 1 ? g.ny : mu == 2 ? g.nz : g.nt;
    const int stride = mu == 1 ? g.hx : mu == 2 ? g.hx * g.ny : g.hx * g.ny * g.nz;
    int n1, n2, n3, n4;
    A s1, s2, s3, s4;
    neighbour<A>(g, i, c, n, stride, mu, +1, n1, s1);
    neighbour<A>(g, i, c, n, stride, mu, -1, n2, s2);
    neighbour<A>(g, i, c, n, stride, mu, +3, n3, s3);
    neighbour<A>(g, i, c, n, stride, mu, -3, n4, s4);
    cplx<A> tmp[NIN][3];
    zero<NIN, A>(tmp);
    const int q = 1 - p;
    HopBuf<NIN, A> b0, b1;
    hop_load<LP, FP, NIN, A, NT>(b0, links + link_block<LP>(0, p, mu, vh), vh, i, in, n1, ncol, r0, nr, 0);
    hop_load<LP, FP, NIN, A, NT>(b1, links + link_block<LP>(0, q, mu, vh), vh, n2, in, n2, ncol, r0, nr, 0);
    hop_apply<LP, NIN, A>(b0, false, s1, nr, tmp, 0);
    hop_load<LP, FP, NIN, A, NT>(b0, links + link_block<LP>(1, p, mu, vh), vh, i, in, n3, ncol, r0, nr, 1);
    hop_apply<LP, NIN, A>(b1, true, s2, nr, tmp, 0);
    hop_load<LP, FP, NIN, A, NT>(b1, links + link_block<LP>(1, q, mu, vh), vh, n4, in, n4, ncol, r0, nr, 1);
    hop_apply<LP, NIN, A>(b0, false, s3, nr, tmp, 1);
    hop_apply<LP, NIN, A>(b1, true, s4, nr, tmp, 1);
    const int par = (mu >= 1 ? s.x : 0) + (mu >= 2 ? s.y : 0) + (mu >= 3 ? s.z : 0);
    const A eta = (par & 1) ? (A)-1 : (A)1;
#pragma unroll
    for (int r = 0; r < NIN; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc[r][a].re = fma(eta, tmp[r][a].re, acc[r][a].re);
            acc[r][a].im = fma(eta, tmp[r][a].im, acc[r][a].im);
        }
}

// Address of hop k (k = 4 mu + {0: +1, 1: -1, 2: +3, 3: -3}) of site s; f:
// the link field (0 fat, 1 Naik).
struct HopAddr {
    const char *blk;
    int ilink, ipsi;
    bool back;
    int f;
};

template <int LP, typename A>
__device__ __forceinline__ HopAddr hop_addr(const Geom &g, int p, const char *links, int i, const Site &s, int k,
                                            A &sg) {
    const int mu = k >> 2, type = k & 3;
    const int c = mu == 0 ? s.x : mu == 1 ? s.y : mu == 2 ? s.z : s.t;
    const int n = mu == 0 ? g.nx : mu == 1 ? g.ny : mu == 2 ? g.nz : g.nt;
    const int stride = mu == 1 ? g.hx : mu == 2 ? g.hx * g.ny : g.hx * g.ny * g.nz;
    const int step = type == 0 ? 1 : type == 1 ? -1 : type == 2 ? 3 : -3;
    int nb;
    neighbour<A>(g, i, c, n, stride, mu, step, nb, sg);
    HopAddr h;
    h.back = (type & 1) != 0;
    const int f = type >> 1;            // 0: fat X (one hop), 1: long W (three hops)
    const int lpar = h.back ? 1 - p : p;
    h.f = f;
    h.blk = links + link_block<LP>(f, lpar, mu, g.vh);
    h.ilink = h.back ? nb : i;
    h.ipsi = nb;
    return h;
}

// acc = (D psi)(site i of parity p), all four directions in this thread.
// The sixteen hops are software-pipelined: the loads of hop k+1 are issued
// before hop k is computed, so two hops' worth of link and vector loads are in
// flight per wavefront instead of one.  The staggered phase eta_mu(s) = +-1 is
// folded into each hop's sign, so every hop accumulates straight into acc
// (summing a direction's four hops apart and then applying eta held 6 NIN more
// accumulators and their zeroing: 16 rhs FP32 NIN 4 216 -> 149 VGPRs, FP64
// NIN 2 256 -> 192; 48^3x12 16 rhs FP16N links 475 -> 439 us, FP64 950 -> 924
// us, 32^3x8 FP64 47.0 -> 46.2 us).
template <int LP, int FP, int NIN, typename A, bool NT, bool ONE = false>
__device__ __forceinline__ void dslash_site(const Geom &g, int p, const char *links, const void *in, int i,
                                            int ncol, int r0, int nr, cplx<A> (&acc)[NIN][3]) {
    const Site s = site_coords(g, p, i);
    zero<NIN, A>(acc);
    auto eta = [&](int k) -> A {  // eta_mu(s) of hop k (mu = k / 4)
        const int mu = k >> 2;
        const int par = (mu >= 1 ? s.x : 0) + (mu >= 2 ? s.y : 0) + (mu >= 3 ? s.z : 0);
        return (par & 1) ? (A)-1 : (A)1;
    };
    if constexpr (NIN > 1) {
        // several right-hand sides: the neighbour vectors two hops ahead, the
        // links one (16 rhs at 48^3x12: FP64 948 -> 918 us, FP32 534 -> 522 us;
        // at one rhs the FP64 kernel was 2 % slower, so it keeps one hop)
        HopBuf<NIN, A> lb[2];
        cplx<A> vb[3][NIN][3];
        A sgv[3];
        bool bkv[3];
        auto load_link = [&](int k, int slot) {
            A sg;
            const HopAddr h = hop_addr<LP, A>(g, p, links, i, s, k, sg);
            LinkIO<LP>::template load<NT>(h.blk, g.vh, h.ilink, lb[slot].m, h.f);
        };
        auto load_vec = [&](int k, int slot) {
            A sg;
            const HopAddr h = hop_addr<LP, A>(g, p, links, i, s, k, sg);
            load_group<FP, NIN, A>(in, g.vh, ncol, r0, nr, h.ipsi, vb[slot]);
            sgv[slot] = sg * eta(k);
            bkv[slot] = h.back;
        };
        load_vec(0, 0);
        load_link(0, 0);
        load_vec(1, 1);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int cur = k & 1, vc = k % 3;
            if (k + 2 < 16)
                load_vec(k + 2, (k + 2) % 3);
            if (k + 1 < 16)
                load_link(k + 1, cur ^ 1);
#pragma unroll
            for (int r = 0; r < NIN; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    lb[cur].v[r][c] = vb[vc][r][c];
            hop_apply<LP, NIN, A>(lb[cur], bkv[vc], sgv[vc], nr, acc, (k & 3) >> 1);
        }
        return;
    }
    HopBuf<NIN, A> buf[2];
    A sgn[2];
    bool back[2];
    auto load = [&](int k, int slot) {
        A sg;
        const HopAddr h = hop_addr<LP, A>(g, p, links, i, s, k, sg);
        LinkIO<LP>::template load<NT>(h.blk, g.vh, h.ilink, buf[slot].m, h.f);
        load_group<FP, NIN, A, ONE>(in, g.vh, ncol, r0, nr, h.ipsi, buf[slot].v);
        sgn[slot] = sg * eta(k);
        back[slot] = h.back;
    };
    load(0, 0);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int cur = k & 1;
        if (k + 1 < 16)
            load(k + 1, cur ^ 1);
        hop_apply<LP, NIN, A, ONE>(buf[cur], back[cur], sgn[cur], nr, acc, (k & 3) >> 1);
    }
}

// prm.ay_rhs[r] (or prm.ay) by static indices: a dynamic index into the
// kernel argument would make the compiler copy the whole argument block to
// scratch memory (280 bytes per lane in the four-lanes-per-site kernel).
__device__ __forceinline__ double ay_of(const DslashParams &prm, int r) {
    double v = prm.ay;
    if (prm.ay_per_rhs) {
#pragma unroll
        for (int q = 0; q < HISQ_MAX_RHS; ++q)
            if (q == r)
                v = prm.ay_rhs[q];
    }
    return v;
}

// out = ad * acc + ay * y  (EPI_AXPY*) for right-hand side r at site i;
// returns Re <y, out> in FP64 (products of the stored-precision values).
// The same with y of the site already loaded (yv; ignored for EPI_PLAIN).
template <int EPI, typename A>
__device__ __forceinline__ double epilogue_y(const DslashParams &prm, int r, const cplx<A> (&yv)[3],
                                             cplx<A> (&v)[3]) {
    double dot = 0.0;
    if (EPI != EPI_PLAIN) {
        const A ad = (A)prm.ad, ay = (A)ay_of(prm, r);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a].re = fma(ad, v[a].re, ay * yv[a].re);
            v[a].im = fma(ad, v[a].im, ay * yv[a].im);
            if (EPI == EPI_AXPY_DOT) {
                dot = fma((double)yv[a].re, (double)v[a].re, dot);
                dot = fma((double)yv[a].im, (double)v[a].im, dot);
            }
        }
    }
    return dot;
}

template <int FP, int EPI, typename A>
__device__ __forceinline__ double epilogue(const DslashParams &prm, int r, int i, cplx<A> (&v)[3]) {
    double dot = 0.0;
    if (EPI != EPI_PLAIN) {
        cplx<A> yv[3];
        FieldIO<FP>::template load<A>(prm.y, prm.g.vh, prm.nrhs, r, i, yv);
        const A ad = (A)prm.ad, ay = (A)ay_of(prm, r);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a].re = fma(ad, v[a].re, ay * yv[a].re);
            v[a].im = fma(ad, v[a].im, ay * yv[a].im);
            if (EPI == EPI_AXPY_DOT) {
                dot = fma((double)yv[a].re, (double)v[a].re, dot);
                dot = fma((double)yv[a].im, (double)v[a].im, dot);
            }
        }
    }
    return dot;
}

// Block partials of the NIN dot products (summed by a finalize kernel).
template <int NIN>
__device__ __forceinline__ void dslash_dot_reduce(const DslashParams &prm, double (&dot)[NIN], const BlockPos<NIN> &bp) {
    __shared__ double lds[4 * NIN];
    block_sum<NIN>(dot, lds);
    if (threadIdx.x == 0)
        for (int r = 0; r < bp.nr; ++r)
            prm.partials[(size_t)(bp.r0 + r) * bp.nsb + bp.sb] = dot[r];
}

// NT: link loads with the non-temporal hint (chosen by the launcher when
// each link is read once: one group of right-hand sides, FP64 or FP32 links).
template <int LP, int FP, int NIN, int EPI, bool NT>
__global__ void __launch_bounds__(256) dslash_site_kernel(const DslashParams prm) {
    constexpr bool ONE = NIN == 1;  // has_col
    using A = typename Prec<LP>::acc;
    if (prm.skip && *prm.skip)
        return;
    const BlockPos<NIN> bp(prm);
    if (!columns_run(prm, bp))
        return;
    const int i = bp.site(prm, bp.sb * blockDim.x + threadIdx.x);
    const bool valid = i < prm.g.vh;
    if (EPI != EPI_AXPY_DOT && !valid)
        return;
    const int r0 = bp.r0, nr = bp.nr;
    double dot[NIN];
#pragma unroll
    for (int r = 0; r < NIN; ++r)
        dot[r] = 0.0;
    if (valid) {
        cplx<A> acc[NIN][3];
        dslash_site<LP, FP, NIN, A, NT, ONE>(prm.g, prm.out_parity, prm.links, prm.in, i, prm.nrhs, r0, nr, acc);
        if constexpr (EPI != EPI_PLAIN) {
            cplx<A> yv[NIN][3];
            load_group<FP, NIN, A>(prm.y, prm.g.vh, prm.nrhs, r0, nr, i, yv);
#pragma unroll
            for (int r = 0; r < NIN; ++r)
                if (r < nr)
                    dot[r] = epilogue_y<EPI, A>(prm, r0 + r, yv[r], acc[r]);
        }
        store_group<FP, NIN, A, ONE>(prm.out, prm.g.vh, prm.nrhs, r0, nr, i, acc);
    }
    if (EPI == EPI_AXPY_DOT)
        dslash_dot_reduce<NIN>(prm, dot, bp);
}

template <int LP, int FP, int NIN, int EPI, bool NT>
__global__ void __launch_bounds__(256) dslash_dir_kernel(const DslashParams prm) {
    using A = typename Prec<LP>::acc;
    if (prm.skip && *prm.skip)
        return;
    const int mu = threadIdx.x & 3;
    const BlockPos<NIN> bp(prm);
    if (!columns_run(prm, bp))
        return;
    const int i = bp.site(prm, bp.sb * (blockDim.x >> 2) + (threadIdx.x >> 2));
    // a site's four lanes are in one wavefront and share validity, so whole
    // quads drop out together and the shuffles below see only valid partners
    const bool valid = i < prm.g.vh;
    if (EPI != EPI_AXPY_DOT && !valid)
        return;
    const int r0 = bp.r0, nr = bp.nr;
    double dot[NIN];
#pragma unroll
    for (int r = 0; r < NIN; ++r)
        dot[r] = 0.0;
    if (valid) {
    const Site s = site_coords(prm.g, prm.out_parity, i);
    // y of the epilogue is loaded with the first hops, not after them
    cplx<A> yv[NIN][3];
    if (EPI != EPI_PLAIN)
        load_group<FP, NIN, A>(prm.y, prm.g.vh, prm.nrhs, r0, nr, i, yv);
    cplx<A> acc[NIN][3];
    zero<NIN, A>(acc);
    dslash_direction<LP, FP, NIN, A, NT>(prm.g, prm.out_parity, prm.links, prm.in, i, s, mu, prm.nrhs, r0, nr,
                                         acc);
    // sum over the quad: (mu0 + mu1) + (mu2 + mu3), identical in all 4 lanes
#pragma unroll
    for (int r = 0; r < NIN; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc[r][a].re += __shfl_xor(acc[r][a].re, 1, 64);
            acc[r][a].im += __shfl_xor(acc[r][a].im, 1, 64);
            acc[r][a].re += __shfl_xor(acc[r][a].re, 2, 64);
            acc[r][a].im += __shfl_xor(acc[r][a].im, 2, 64);
        }
#pragma unroll
    for (int r = 0; r < NIN; ++r) {
        if (r < nr) {
            const double d = epilogue_y<EPI, A>(prm, r0 + r, yv[r], acc[r]);
            dot[r] = mu == 0 ? d : 0.0;  // one lane of the quad counts the site
        }
    }
    if constexpr (FP == HISQ_FP16N) {
#pragma unroll
        for (int r = 0; r < NIN; ++r)
            if (r < nr && mu == 0)  // one 16-byte record holds the whole site
                FieldIO<FP>::template store<A>(prm.out, prm.g.vh, prm.nrhs, r0 + r, i, acc[r]);
    } else if constexpr (FP == HISQ_FP32 && NIN % 2 == 0) {
        // lane mu < 3 writes colour mu of both slots of each pair (the unused
        // slot of an odd last column gets zero)
#pragma unroll
        for (int r = 0; r < NIN; r += 2)
            if (r < nr) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (mu == c)
                        FieldIO<FP>::template store_colour_pair<A>(prm.out, prm.g.vh, (r0 + r) >> 1, i, c, acc[r][c],
                                                                   acc[r + 1][c]);
            }
    } else {
        // lane mu < 3 writes colour mu (static indices keep acc in registers)
#pragma unroll
        for (int r = 0; r < NIN; ++r)
            if (r < nr) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (mu == c)
                        FieldIO<FP>::template store_colour<A>(prm.out, prm.g.vh, prm.nrhs, r0 + r, i, c, acc[r][c]);
            }
    }
    }
    if (EPI == EPI_AXPY_DOT)
        dslash_dot_reduce<NIN>(prm, dot, bp);
}

// Sixteen lanes per output site (VAR_HOP), lane k computing hop k alone (its
// link and neighbour vectors: one round of loads), the sixteen partial
// results combined by four butterfly shuffles within the group.  For lattices
// too small to fill the GPU with one thread or four lanes per site, where each
// launch is bound by the latency of its chain of loads.  NIN <= 2.
template <int LP, int FP, int NIN, int EPI, bool NT>
__global__ void __launch_bounds__(256) dslash_hop_kernel(const DslashParams prm) {
    using A = typename Prec<LP>::acc;
    if (prm.skip && *prm.skip)
        return;
    const BlockPos<NIN> bp(prm);
    if (!columns_run(prm, bp))
        return;
    const int k = threadIdx.x & 15;
    const int i = bp.site(prm, bp.sb * (blockDim.x >> 4) + (threadIdx.x >> 4));
    // a site's sixteen lanes share validity, so whole groups drop out together
    const bool valid = i < prm.g.vh;
    if (EPI != EPI_AXPY_DOT && !valid)
        return;
    const int r0 = bp.r0, nr = bp.nr;
    double dot[NIN];
#pragma unroll
    for (int r = 0; r < NIN; ++r)
        dot[r] = 0.0;
    if (valid) {
        const Geom &g = prm.g;
        const int p = prm.out_parity;
        const Site s = site_coords(g, p, i);
        A sg;
        const HopAddr h = hop_addr<LP, A>(g, p, prm.links, i, s, k, sg);
        HopBuf<NIN, A> b;
        LinkIO<LP>::template load<NT>(h.blk, g.vh, h.ilink, b.m, h.f);
#pragma unroll
        for (int r = 0; r < NIN; ++r)
            if (r < nr)
                FieldIO<FP>::template load<A>(prm.in, g.vh, prm.nrhs, r0 + r, h.ipsi, b.v[r]);
        cplx<A> yv[NIN][3];
        if (EPI != EPI_PLAIN) {
#pragma unroll
            for (int r = 0; r < NIN; ++r)
                if (r < nr)
                    FieldIO<FP>::template load<A>(prm.y, g.vh, prm.nrhs, r0 + r, i, yv[r]);
        }
        cplx<A> acc[NIN][3];
        zero<NIN, A>(acc);
        hop_apply<LP, NIN, A>(b, h.back, sg, nr, acc, h.f);
        const int mu = k >> 2;
        const int par = (mu >= 1 ? s.x : 0) + (mu >= 2 ? s.y : 0) + (mu >= 3 ? s.z : 0);
        const A eta = (par & 1) ? (A)-1 : (A)1;
        // sum over the group: ((k ^ 1) + ...) in a fixed butterfly, identical in all 16 lanes
#pragma unroll
        for (int r = 0; r < NIN; ++r)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                A re = eta * acc[r][a].re, im = eta * acc[r][a].im;
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) {
                    re += __shfl_xor(re, o, 64);
                    im += __shfl_xor(im, o, 64);
                }
                acc[r][a].re = re;
                acc[r][a].im = im;
            }
#pragma unroll
        for (int r = 0; r < NIN; ++r) {
            if (r < nr) {
                const double d = epilogue_y<EPI, A>(prm, r0 + r, yv[r], acc[r]);
                dot[r] = k == 0 ? d : 0.0;  // one lane of the group counts the site
                if constexpr (FP == HISQ_FP16N) {
                    if (k == 0)
                        FieldIO<FP>::template store<A>(prm.out, g.vh, prm.nrhs, r0 + r, i, acc[r]);
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        if (k == c)
                            FieldIO<FP>::template store_colour<A>(prm.out, g.vh, prm.nrhs, r0 + r, i, c, acc[r][c]);
                }
            }
        }
    }
    if (EPI == EPI_AXPY_DOT)
        dslash_dot_reduce<NIN>(prm, dot, bp);
}

// ---------------------------------------------------------------------------
// LDS-staged neighbours (VAR_LDS), for several right-hand sides in the banded
// z-slab block order: a block is one piece of LDS_BAND y-rows x N_x/2 sites at
// fixed (t, z), one thread per site.  The block first copies, for its group of
// right-hand sides, the input rows y0 - 3 .. y0 + LDS_BAND + 2 of that (t, z)
// (the rows every x- and y-hop of the piece reads) into LDS with coalesced
// loads; the eight x- and y-hops then read their neighbour vectors from LDS,
// the z- and t-hops through the caches.  Each staged vector serves up to eight
// hops of the piece, so the vector loads issued per site fall from 16 NIN x 3
// to 8 NIN x 3 plus (1 + 6 / LDS_BAND) NIN x 3 for the staging.
// ---------------------------------------------------------------------------
constexpr int LDS_BAND = 8;
constexpr int LDS_HALO = 3;

template <int FP> struct StageElem;
template <> struct StageElem<HISQ_FP64> { using T = double2; };
template <> struct StageElem<HISQ_FP32> { using T = float2; };

// Bytes of LDS a VAR_LDS block needs for nin right-hand sides.
__host__ __device__ inline size_t lds_stage_bytes(const Geom &g, int fp, int nin) {
    return (size_t)nin * 3 * (LDS_BAND + 2 * LDS_HALO) * g.hx * (fp == HISQ_FP64 ? 16 : 8);
}

template <int LP, int FP, int NIN, int EPI, bool NT>
__global__ void __launch_bounds__(256) dslash_lds_kernel(const DslashParams prm) {
    using A = typename Prec<LP>::acc;
    using E = typename StageElem<FP>::T;
    extern __shared__ char lds_raw[];
    E *stage = reinterpret_cast<E *>(lds_raw);
    if (prm.skip && *prm.skip)
        return;
    const BlockPos<NIN> bp(prm);
    if (!columns_run(prm, bp))
        return;
    const Geom &g = prm.g;
    const int p = prm.out_parity;
    // the piece: (t, z, y-band) of the banded z-slab traversal, q = bp.sb
    const int zw = g.nz >> 3;
    const int q = bp.sb;
    const int zl = q % zw;
    int st = q / zw;
    const int t = st % g.nt;
    st /= g.nt;
    const int nbands = g.ny / LDS_BAND;
    const int bd = st % nbands, slab = st / nbands;
    const int z = slab * zw + zl;
    const int y0 = bd * LDS_BAND;
    const int plane = (t * g.nz + z) * (g.ny * g.hx);  // half index of (t, z, y = 0, xh = 0)
    const int nrow = LDS_BAND + 2 * LDS_HALO;
    const int r0 = bp.r0, nr = bp.nr;
    // stage rows y0 - 3 .. y0 + band + 2 (periodic in y) of the input parity:
    // blockDim = LDS_BAND * hx threads and NIN * 3 * nrow * hx elements, so
    // each thread copies at most PER of them; all its loads are issued
    // before the first LDS store
    // FP32 fields with NIN even: whole column pairs, one 16-byte record per
    // (pair, colour, site), staged as such
    constexpr bool PAIRS = FP == HISQ_FP32 && NIN % 2 == 0;
    if constexpr (PAIRS) {
        constexpr int PER = ((NIN / 2) * 3 * (LDS_BAND + 2 * LDS_HALO) + LDS_BAND - 1) / LDS_BAND;
        const int per_rc = nrow * g.hx;
        const int total = ((nr + 1) / 2) * 3 * per_rc;
        const nt_f4 *src = reinterpret_cast<const nt_f4 *>(prm.in);
        nt_f4 *stage4 = reinterpret_cast<nt_f4 *>(lds_raw);
        nt_f4 v[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            // past the staged records: the group's first record, loaded and
            // not stored (unconditional loads keep v in registers)
            const int e0 = threadIdx.x + j * blockDim.x;
            const int e = e0 < total ? e0 : 0;
            const int pc = e / per_rc, rem = e - pc * per_rc;
            const int row = rem / g.hx, xh = rem - row * g.hx;
            int gy = y0 - LDS_HALO + row;
            gy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
            v[j] = src[((size_t)(r0 / 2) * 3 + pc) * g.vh + plane + gy * g.hx + xh];
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + j * blockDim.x;
            if (e < total)
                stage4[e] = v[j];
        }
    } else {
        constexpr int PER = (NIN * 3 * (LDS_BAND + 2 * LDS_HALO) + LDS_BAND - 1) / LDS_BAND;
        const int per_rc = nrow * g.hx;
        const int total = nr * 3 * per_rc;
        const E *src = reinterpret_cast<const E *>(prm.in);
        E v[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            // past the staged elements: the group's first element, loaded and
            // not stored (unconditional loads keep v in registers)
            const int e0 = threadIdx.x + j * blockDim.x;
            const int e = e0 < total ? e0 : 0;
            const int rc = e / per_rc, rem = e - rc * per_rc;
            const int row = rem / g.hx, xh = rem - row * g.hx;
            int gy = y0 - LDS_HALO + row;
            gy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
            const int site = plane + gy * g.hx + xh;
            if constexpr (FP == HISQ_FP32)
                v[j] = src[f32_index(g.vh, prm.nrhs, r0 + rc / 3, rc % 3, site)];
            else
                v[j] = src[(size_t)(r0 * 3 + rc) * g.vh + site];
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + j * blockDim.x;
            if (e < total)
                stage[e] = v[j];
        }
    }
    __syncthreads();
    const int ry = threadIdx.x / g.hx, xh = threadIdx.x - ry * g.hx;
    const int y = y0 + ry;
    const int i = plane + y * g.hx + xh;
    Site s;
    s.y = y;
    s.z = z;
    s.t = t;
    s.x = 2 * xh + ((y + z + t + p) & 1);
    cplx<A> acc[NIN][3];
    zero<NIN, A>(acc);
    auto eta = [&](int k) -> A {  // eta_mu(s) of hop k, folded into its sign
        const int mu = k >> 2;
        const int par = (mu >= 1 ? s.x : 0) + (mu >= 2 ? s.y : 0) + (mu >= 3 ? s.z : 0);
        return (par & 1) ? (A)-1 : (A)1;
    };
    HopBuf<NIN, A> buf[2];
    A sgn[2];
    bool back[2];
    auto load = [&](int k, int slot) {
        A sg;
        const HopAddr h = hop_addr<LP, A>(g, p, prm.links, i, s, k, sg);
        LinkIO<LP>::template load<NT>(h.blk, g.vh, h.ilink, buf[slot].m, h.f);
        const int mu = k >> 2;
        if (mu >= 2) {
            load_group<FP, NIN, A>(prm.in, g.vh, prm.nrhs, r0, nr, h.ipsi, buf[slot].v);
        } else {
            // LDS row and column of the neighbour: x-hops stay in the row,
            // y-hops move rows (the staged rows start at y0 - 3)
            const int type = k & 3;
            const int step = type == 0 ? 1 : type == 1 ? -1 : type == 2 ? 3 : -3;
            int row = ry + LDS_HALO, col = xh;
            if (mu == 1) {
                row += step;
            } else {
                int xn = s.x + step;
                xn = xn < 0 ? xn + g.nx : (xn >= g.nx ? xn - g.nx : xn);
                col = xn >> 1;
            }
            if constexpr (PAIRS) {
                // every pair slot of the buffer is read (the ones past the
                // group's columns hold stale values that are never used),
                // which keeps the vectors in registers
                const nt_f4 *stage4 = reinterpret_cast<const nt_f4 *>(lds_raw);
#pragma unroll
                for (int r = 0; r < NIN; r += 2) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const nt_f4 e = stage4[(((r >> 1) * 3 + c) * nrow + row) * g.hx + col];
                        buf[slot].v[r][c].re = (A)e.x;
                        buf[slot].v[r][c].im = (A)e.y;
                        buf[slot].v[r + 1][c].re = (A)e.z;
                        buf[slot].v[r + 1][c].im = (A)e.w;
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < NIN; ++r) {
                    if (r < nr) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const E e = stage[((r * 3 + c) * nrow + row) * g.hx + col];
                            buf[slot].v[r][c].re = (A)e.x;
                            buf[slot].v[r][c].im = (A)e.y;
                        }
                    }
                }
            }
        }
        sgn[slot] = sg * eta(k);
        back[slot] = h.back;
    };
    load(0, 0);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int cur = k & 1;
        if (k + 1 < 16)
            load(k + 1, cur ^ 1);
        hop_apply<LP, NIN, A>(buf[cur], back[cur], sgn[cur], nr, acc, (k & 3) >> 1);
    }
    double dot[NIN];
#pragma unroll
    for (int r = 0; r < NIN; ++r)
        dot[r] = 0.0;
    if constexpr (EPI != EPI_PLAIN) {
        cplx<A> yv[NIN][3];
        load_group<FP, NIN, A>(prm.y, g.vh, prm.nrhs, r0, nr, i, yv);
#pragma unroll
        for (int r = 0; r < NIN; ++r)
            if (r < nr)
                dot[r] = epilogue_y<EPI, A>(prm, r0 + r, yv[r], acc[r]);
    }
    store_group<FP, NIN, A>(prm.out, g.vh, prm.nrhs, r0, nr, i, acc);
    if (EPI == EPI_AXPY_DOT)
        dslash_dot_reduce<NIN>(prm, dot, bp);
}

}  // namespace hisq
