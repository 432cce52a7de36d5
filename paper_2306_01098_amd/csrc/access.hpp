// Device loads and stores of packed links and colour-vector fields.
#pragma once

#include "common.hpp"

namespace hisq {

// ---------------------------------------------------------------------------
// Link matrices: 18 reals, row-major, (re, im) interleaved.
// ---------------------------------------------------------------------------
template <int LP> struct LinkIO;

// With one group of right-hand sides every link is read exactly once per
// Dslash application, and FP64, FP32 and W14 link loads may carry the
// non-temporal hint (stream = true; NT = true): they stream through the caches
// without displacing the neighbour vectors, which are reused up to 16 times.
// The launcher gives it only where the link set of one application (both
// parities' blocks) exceeds the 256 MiB MALL, where ordinary loads would cache
// nothing for the next application (32^3x8 FP64, 302 MB: D_oe and D_eo
// alternating 51.0 -> 49.4 us with the hint, the FP64 CG 18.3 -> 16.7 ms;
// 16 single FP32 solves at 48^3x12, 764 MB: 1.43 -> 1.34 s).  Smaller link
// sets are read with ordinary loads and partly come from the MALL (32^3x8 FP32,
// 151 MB: 26.3 -> 24.6 us, the FP32 CG 10.96 -> 10.44 ms; FP64W14, 256 MiB:
// 47.3 -> 45.3 us; FP32W14 24.6 -> 22.2 us).  When N_outer > 1 groups of
// right-hand sides read the same links one after another, the links must stay
// in the L2 for the next group, and ordinary loads are faster (16 rhs at
// 48^3x12: FP64 1113 -> 960 us, FP32 576 -> 533 us); so are they for
// reconstruct-12 links at any N_outer (32^3x8 FP64R12 35.4 -> 33.7 us) and for
// binary16 links.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));

template <bool NT, typename V> __device__ __forceinline__ V ld_link(const V *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <> struct LinkIO<HISQ_FP64> {
    using A = double;
    static constexpr bool rebuild = false;
    __device__ __forceinline__ static void finish(A *, int) {}
    static constexpr bool stream = true;  // the non-temporal hint may pay
    template <bool NT = true>
    __device__ __forceinline__ static void load(const char *blk, int vh, int i, A m[18], int f = 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const nt_d2 v = ld_link<NT>(reinterpret_cast<const nt_d2 *>(blk + (size_t)vh * 16 * k) + i);
            m[2 * k] = v.x;
            m[2 * k + 1] = v.y;
        }
    }
};

template <> struct LinkIO<HISQ_FP32> {
    using A = float;
    static constexpr bool rebuild = false;
    __device__ __forceinline__ static void finish(A *, int) {}
    static constexpr bool stream = true;  // the non-temporal hint may pay
    template <bool NT = true>
    __device__ __forceinline__ static void load(const char *blk, int vh, int i, A m[18], int f = 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const nt_f4 v = ld_link<NT>(reinterpret_cast<const nt_f4 *>(blk + (size_t)vh * 16 * k) + i);
            m[4 * k] = v.x;
            m[4 * k + 1] = v.y;
            m[4 * k + 2] = v.z;
            m[4 * k + 3] = v.w;
        }
        const nt_f2 t = ld_link<NT>(reinterpret_cast<const nt_f2 *>(blk + (size_t)vh * 64) + i);
        m[16] = t.x;
        m[17] = t.y;
    }
};

union H8 {
    uint4 u;
    _Float16 h[8];
};
union H2 {
    uint32_t u;
    _Float16 h[2];
};

template <> struct LinkIO<HISQ_FP16N> {
    using A = float;
    static constexpr bool rebuild = false;
    __device__ __forceinline__ static void finish(A *, int) {}
    static constexpr bool stream = false;  // ordinary loads at any size
    template <bool NT = true>  // ordinary loads either way
    __device__ __forceinline__ static void load(const char *blk, int vh, int i, A m[18], int f = 0) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            H8 v;
            v.u = reinterpret_cast<const uint4 *>(blk + (size_t)vh * 16 * k)[i];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                m[8 * k + j] = (float)v.h[j];
        }
        H2 t;
        t.u = reinterpret_cast<const uint32_t *>(blk + (size_t)vh * 32)[i];
        m[16] = (float)t.h[0];
        m[17] = (float)t.h[1];
    }
};

template <typename A> __device__ __forceinline__ void rebuild_row2(A m[18]);
template <typename A> __device__ __forceinline__ void rebuild_row2_scaled(A m[18]);

// Reconstruct-12: load fills m[0..11] (rows 0 and 1); finish (rebuild_row2)
// computes row 2 at the point of use, so the loads of the next hop stay in
// flight.
template <> struct LinkIO<HISQ_FP64R12> {
    using A = double;
    static constexpr bool rebuild = true;
    __device__ __forceinline__ static void finish(A *m, int) { rebuild_row2<A>(m); }
    static constexpr bool stream = false;  // ordinary loads at any size
    template <bool NT = true>
    __device__ __forceinline__ static void load(const char *blk, int vh, int i, A m[18], int f = 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const nt_d2 v = ld_link<NT>(reinterpret_cast<const nt_d2 *>(blk + (size_t)vh * 16 * k) + i);
            m[2 * k] = v.x;
            m[2 * k + 1] = v.y;
        }
    }
};

template <> struct LinkIO<HISQ_FP32R12> {
    using A = float;
    static constexpr bool rebuild = true;
    __device__ __forceinline__ static void finish(A *m, int) { rebuild_row2<A>(m); }
    static constexpr bool stream = false;  // ordinary loads at any size
    template <bool NT = true>
    __device__ __forceinline__ static void load(const char *blk, int vh, int i, A m[18], int f = 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const nt_f4 v = ld_link<NT>(reinterpret_cast<const nt_f4 *>(blk + (size_t)vh * 16 * k) + i);
            m[4 * k] = v.x;
            m[4 * k + 1] = v.y;
            m[4 * k + 2] = v.z;
            m[4 * k + 3] = v.w;
        }
    }
};

// W14: fat links (f = 0) in full as HISQ_FP64 / HISQ_FP32; Naik links
// (f = 1) as rows 0 and 1 and the factor z = (m[12], m[13]), row 2 rebuilt
// by finish as z conj(row 0 x row 1).
template <> struct LinkIO<HISQ_FP64W14> {
    using A = double;
    static constexpr bool rebuild = true;
    static constexpr bool stream = true;  // the non-temporal hint may pay
    __device__ __forceinline__ static void finish(A *m, int f) {
        if (f == 1)
            rebuild_row2_scaled<A>(m);
    }
    template <bool NT = true>
    __device__ __forceinline__ static void load(const char *blk, int vh, int i, A m[18], int f = 0) {
        const int nc = f == 0 ? 9 : 7;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            if (k < nc) {
                const nt_d2 v = ld_link<NT>(reinterpret_cast<const nt_d2 *>(blk + (size_t)vh * 16 * k) + i);
                m[2 * k] = v.x;
                m[2 * k + 1] = v.y;
            }
        }
    }
};

template <> struct LinkIO<HISQ_FP32W14> {
    using A = float;
    static constexpr bool rebuild = true;
    static constexpr bool stream = true;  // the non-temporal hint may pay
    __device__ __forceinline__ static void finish(A *m, int f) {
        if (f == 1)
            rebuild_row2_scaled<A>(m);
    }
    template <bool NT = true>
    __device__ __forceinline__ static void load(const char *blk, int vh, int i, A m[18], int f = 0) {
        const int nc = f == 0 ? 4 : 3;  // 16-byte chunks before the 8-byte tail
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < nc) {
                const nt_f4 v = ld_link<NT>(reinterpret_cast<const nt_f4 *>(blk + (size_t)vh * 16 * k) + i);
                m[4 * k] = v.x;
                m[4 * k + 1] = v.y;
                m[4 * k + 2] = v.z;
                m[4 * k + 3] = v.w;
            }
        }
        // tail: entries 16, 17 of a full matrix, or the factor z of a Naik link
        const nt_f2 t = ld_link<NT>(reinterpret_cast<const nt_f2 *>(blk + (size_t)vh * 16 * nc) + i);
        m[f == 0 ? 16 : 12] = t.x;
        m[f == 0 ? 17 : 13] = t.y;
    }
};

// Row 2 of a special-unitary matrix from rows 0 (a) and 1 (b): since
// det U = 1 and U^+ = U^-1, row 2 = conj(a x b), i.e.
// c_k = conj(a_{k+1} b_{k+2} - a_{k+2} b_{k+1}) (indices mod 3).
template <typename A> __device__ __forceinline__ void rebuild_row2(A m[18]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int j = (k + 1) % 3, l = (k + 2) % 3;
        const A ajr = m[2 * j], aji = m[2 * j + 1], alr = m[2 * l], ali = m[2 * l + 1];
        const A bjr = m[6 + 2 * j], bji = m[6 + 2 * j + 1], blr = m[6 + 2 * l], bli = m[6 + 2 * l + 1];
        // a_j b_l - a_l b_j
        const A re = fma(ajr, blr, fma(-aji, bli, fma(-alr, bjr, ali * bji)));
        const A im = fma(ajr, bli, fma(aji, blr, fma(-alr, bji, -ali * bjr)));
        m[12 + 2 * k] = re;
        m[12 + 2 * k + 1] = -im;
    }
}

// Row 2 = z conj(a x b) with z = (m[12], m[13]) (read before row 2 is
// written over it): exact for real multiples of U(3) matrices.
template <typename A> __device__ __forceinline__ void rebuild_row2_scaled(A m[18]) {
    const A zr = m[12], zi = m[13];
    rebuild_row2<A>(m);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const A cr = m[12 + 2 * k], ci = m[12 + 2 * k + 1];
        m[12 + 2 * k] = fma(zr, cr, -zi * ci);
        m[12 + 2 * k + 1] = fma(zr, ci, zi * cr);
    }
}

// ---------------------------------------------------------------------------
// Colour-vector fields on one parity.  Every access names the column count n
// of the packed field it reads (a sequence of one-column fields laid end to
// end, such as the shifted directions of the multi-shift solver or the PTC
// channels, is addressed with n = 1).
//   FP64: [column][colour][site] of 16-byte {re, im}.
//   FP32, n = 1: [colour][site] of 8-byte {re, im}.
//   FP32, n >= 2: columns 2j and 2j + 1 share 16-byte records {re, im of
//     column 2j, re, im of column 2j + 1}, [pair][colour][site], so that a
//     thread holding both columns of a pair issues one 16-byte load per colour
//     instead of two 8-byte ones; for odd n the second slot of the last pair
//     is unused (the field takes 24 (n + 1) bytes per site), so every column
//     of the field belongs to a pair and the first 2k columns are laid out as
//     a 2k-column field.
//   FP16N: one 16-byte record per site and column, [column][site].
// ---------------------------------------------------------------------------

// Index, in 8-byte {re, im} units, of colour c of site i of column r of an
// n-column FP32 field.
__host__ __device__ __forceinline__ size_t f32_index(int vh, int n, int r, int c, int i) {
    if (n >= 2)
        return (((size_t)(r >> 1) * 3 + c) * vh + i) * 2 + (r & 1);
    return ((size_t)r * 3 + c) * vh + i;
}

template <int FP> struct FieldIO;

template <> struct FieldIO<HISQ_FP64> {
    template <typename A>
    __device__ __forceinline__ static void load(const void *f, int vh, int n, int r, int i, cplx<A> v[3]) {
        (void)n;
        const double2 *p = reinterpret_cast<const double2 *>(f) + (size_t)r * 3 * vh + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double2 d = p[(size_t)c * vh];
            v[c].re = (A)d.x;
            v[c].im = (A)d.y;
        }
    }
    // FP64 results are stored with the non-temporal hint: a written value is
    // not read again by the same launch, and keeping it out of the L2 leaves
    // room for the neighbour vectors (32^3x8 FP64 Dslash 50.0 -> 48.8-49.2 us,
    // FP64 CG 18.55 -> 18.14 ms; FP32 stores showed no gain and stay plain).
    template <typename A>
    __device__ __forceinline__ static void store(void *f, int vh, int n, int r, int i, const cplx<A> v[3]) {
        (void)n;
        nt_d2 *p = reinterpret_cast<nt_d2 *>(f) + (size_t)r * 3 * vh + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            nt_d2 t;
            t.x = (double)v[c].re;
            t.y = (double)v[c].im;
            __builtin_nontemporal_store(t, p + (size_t)c * vh);
        }
    }
    template <typename A>
    __device__ __forceinline__ static void store_colour(void *f, int vh, int n, int r, int i, int c, cplx<A> v) {
        (void)n;
        nt_d2 t;
        t.x = (double)v.re;
        t.y = (double)v.im;
        __builtin_nontemporal_store(t, reinterpret_cast<nt_d2 *>(f) + ((size_t)r * 3 + c) * vh + i);
    }
};

template <> struct FieldIO<HISQ_FP32> {
    template <typename A>
    __device__ __forceinline__ static void load(const void *f, int vh, int n, int r, int i, cplx<A> v[3]) {
        const float2 *p = reinterpret_cast<const float2 *>(f);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float2 d = p[f32_index(vh, n, r, c, i)];
            v[c].re = (A)d.x;
            v[c].im = (A)d.y;
        }
    }
    template <typename A>
    __device__ __forceinline__ static void store(void *f, int vh, int n, int r, int i, const cplx<A> v[3]) {
        float2 *p = reinterpret_cast<float2 *>(f);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            p[f32_index(vh, n, r, c, i)] = make_float2((float)v[c].re, (float)v[c].im);
    }
    template <typename A>
    __device__ __forceinline__ static void store_colour(void *f, int vh, int n, int r, int i, int c, cplx<A> v) {
        reinterpret_cast<float2 *>(f)[f32_index(vh, n, r, c, i)] = make_float2((float)v.re, (float)v.im);
    }
    // Both slots of pair j (columns 2j and 2j + 1) of a multi-column field:
    // one 16-byte access per colour.
    template <typename A>
    __device__ __forceinline__ static void load_pair(const void *f, int vh, int j, int i, cplx<A> v0[3],
                                                     cplx<A> v1[3]) {
        const float4 *p = reinterpret_cast<const float4 *>(f) + (size_t)j * 3 * vh + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float4 d = p[(size_t)c * vh];
            v0[c].re = (A)d.x;
            v0[c].im = (A)d.y;
            v1[c].re = (A)d.z;
            v1[c].im = (A)d.w;
        }
    }
    template <typename A>
    __device__ __forceinline__ static void store_colour_pair(void *f, int vh, int j, int i, int c, cplx<A> v0,
                                                             cplx<A> v1) {
        reinterpret_cast<float4 *>(f)[((size_t)j * 3 + c) * vh + i] =
            make_float4((float)v0.re, (float)v0.im, (float)v1.re, (float)v1.im);
    }
    template <typename A>
    __device__ __forceinline__ static void store_pair(void *f, int vh, int j, int i, const cplx<A> v0[3],
                                                      const cplx<A> v1[3]) {
        float4 *p = reinterpret_cast<float4 *>(f) + (size_t)j * 3 * vh + i;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            p[(size_t)c * vh] = make_float4((float)v0[c].re, (float)v0[c].im, (float)v1[c].re, (float)v1[c].im);
    }
};

// binary16 components scaled by a binary32 per-site norm, one 16-byte record
// per site: {re0, im0, re1, im1, re2, im2} halves, then the float norm.
union F16NRecord {
    uint4 u;
    struct {
        _Float16 h[6];
        float norm;
    } s;
};

template <> struct FieldIO<HISQ_FP16N> {
    template <typename A>
    __device__ __forceinline__ static void load(const void *f, int vh, int ncol, int r, int i, cplx<A> v[3]) {
        (void)ncol;
        F16NRecord rec;
        rec.u = reinterpret_cast<const uint4 *>(f)[(size_t)r * vh + i];
        const float n = rec.s.norm;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c].re = (A)((float)rec.s.h[2 * c] * n);
            v[c].im = (A)((float)rec.s.h[2 * c + 1] * n);
        }
    }
    // Norm n = max |component| (exact in FP32); components stored as
    // binary16(v / n) with the division in FP32.
    template <typename A>
    __device__ __forceinline__ static void store(void *f, int vh, int ncol, int r, int i, const cplx<A> v[3]) {
        (void)ncol;
        float x[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[2 * c] = (float)v[c].re;
            x[2 * c + 1] = (float)v[c].im;
        }
        float n = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            n = fmaxf(n, fabsf(x[k]));
        F16NRecord rec;
        const float inv_ok = n > 0.f ? 1.f : 0.f;
        const float d = n > 0.f ? n : 1.f;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            rec.s.h[k] = (_Float16)(inv_ok * (x[k] / d));
        rec.s.norm = n;
        reinterpret_cast<uint4 *>(f)[(size_t)r * vh + i] = rec.u;
    }
};

}  // namespace hisq
