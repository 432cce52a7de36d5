// Shared device/host definitions of the gfx950 HISQ library: packed layouts,
// lattice index helpers and small complex arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "hisq.h"

namespace hisq {

// ---------------------------------------------------------------------------
// Lattice geometry on the device.  A site of parity p with coordinates
// (x, y, z, t) has half-lattice index i = floor(lex / 2) with
// lex = x + Nx (y + Ny (z + Nz t)) (the even/odd memory order of Sec. 4.3);
// because Nx is even, i = x/2 + (Nx/2) (y + Ny (z + Nz t)).
// ---------------------------------------------------------------------------
struct Geom {
    int nx, ny, nz, nt;  // extents
    int hx;              // nx / 2
    int vh;              // V / 2 sites per parity
    int t_bc;            // +1 / -1 time boundary sign of colour vectors
};

inline Geom make_geom(const hisq_lattice &l) {
    Geom g;
    g.nx = l.dims[0];
    g.ny = l.dims[1];
    g.nz = l.dims[2];
    g.nt = l.dims[3];
    g.hx = g.nx / 2;
    g.vh = (int)((int64_t)g.nx * g.ny * g.nz * g.nt / 2);
    g.t_bc = l.t_bc;
    return g;
}

// ---------------------------------------------------------------------------
// Packed link layout.  For each field f (0 = X fat, 1 = W long), parity p of
// the site the link leaves from, and direction mu, one block of vh matrices.
// A block stores the 18 reals of each matrix (row-major, re/im interleaved)
// split into 16-byte chunks, structure of arrays: chunk k of all vh sites is
// contiguous, so a wavefront reading chunk k for 64 consecutive sites issues
// one fully coalesced 1 KiB request.  The last chunk may be shorter
// (FP32: 8 bytes, FP16: 4 bytes).  Reconstruct-12 formats store only the 12
// reals of rows 0 and 1 (FP64: 6 chunks, FP32: 3 chunks).  The W14 formats
// store the fat links X in full and the Naik links W as rows 0 and 1 plus a
// complex factor z (14 reals: FP64 7 chunks, FP32 3 chunks + 8 bytes); all X
// blocks come first, then the W blocks.
// ---------------------------------------------------------------------------
template <int P> struct Prec;
template <> struct Prec<HISQ_FP64> {
    using store = double;
    using acc = double;
    static constexpr int real_bytes = 8;
    static constexpr int mat_bytes = 18 * 8;
};
template <> struct Prec<HISQ_FP32> {
    using store = float;
    using acc = float;
    static constexpr int real_bytes = 4;
    static constexpr int mat_bytes = 18 * 4;
};
template <> struct Prec<HISQ_FP16N> {
    using store = _Float16;
    using acc = float;
    static constexpr int real_bytes = 2;
    static constexpr int mat_bytes = 18 * 2;
};
// Reconstruct-12 links: rows 0 and 1 stored (12 reals), row 2 rebuilt.
template <> struct Prec<HISQ_FP64R12> {
    using store = double;
    using acc = double;
    static constexpr int real_bytes = 8;
    static constexpr int mat_bytes = 12 * 8;
};
template <> struct Prec<HISQ_FP32R12> {
    using store = float;
    using acc = float;
    static constexpr int real_bytes = 4;
    static constexpr int mat_bytes = 12 * 4;
};
// W14: mat_bytes is the fat-link matrix, mat_bytes_w the Naik-link matrix.
template <> struct Prec<HISQ_FP64W14> {
    using store = double;
    using acc = double;
    static constexpr int real_bytes = 8;
    static constexpr int mat_bytes = 18 * 8;
    static constexpr int mat_bytes_w = 14 * 8;
};
template <> struct Prec<HISQ_FP32W14> {
    using store = float;
    using acc = float;
    static constexpr int real_bytes = 4;
    static constexpr int mat_bytes = 18 * 4;
    static constexpr int mat_bytes_w = 14 * 4;
};

// Bytes of one stored fat-link (X) and Naik-link (W) matrix, and the
// precision of the colour-vector fields that go with a link precision.
__host__ __device__ constexpr int link_matrix_bytes(int prec) {
    return prec == HISQ_FP64 ? 144 : prec == HISQ_FP32 ? 72 : prec == HISQ_FP16N ? 36
         : prec == HISQ_FP64R12 ? 96 : prec == HISQ_FP32R12 ? 48 : prec == HISQ_FP64W14 ? 144 : 72;
}
__host__ __device__ constexpr int link_matrix_bytes_w(int prec) {
    return prec == HISQ_FP64W14 ? 112 : prec == HISQ_FP32W14 ? 56 : link_matrix_bytes(prec);
}
__host__ __device__ constexpr int field_prec_of(int prec) {
    return prec == HISQ_FP64R12 || prec == HISQ_FP64W14   ? HISQ_FP64
           : prec == HISQ_FP32R12 || prec == HISQ_FP32W14 ? HISQ_FP32
                                                          : prec;
}

inline size_t links_bytes(const Geom &g, int prec) {
    return (size_t)2 * 4 * (size_t)g.vh * (link_matrix_bytes(prec) + link_matrix_bytes_w(prec));
}

// Byte offset of the block (f, p, mu) for fat-link matrices of mx bytes and
// Naik-link matrices of mw bytes (all X blocks first).
__host__ __device__ inline size_t link_block(int f, int p, int mu, int vh, int mx, int mw) {
    return f == 0 ? (size_t)(p * 4 + mu) * (size_t)vh * mx
                  : (size_t)8 * vh * mx + (size_t)(p * 4 + mu) * (size_t)vh * mw;
}
template <int LP> __host__ __device__ inline size_t link_block(int f, int p, int mu, int vh) {
    return link_block(f, p, mu, vh, link_matrix_bytes(LP), link_matrix_bytes_w(LP));
}

// ---------------------------------------------------------------------------
// Packed field layout (one parity, nrhs right-hand sides).
//   FP64:  [rhs][colour][site] complex (16 bytes per element).
//   FP32:  one column [colour][site] complex (8 bytes per element); two or
//          more columns in pairs, [pair][colour][site] 16-byte records (the
//          second slot of the last pair unused when nrhs is odd).
//   FP16N: [rhs][site] 16-byte records {half2 c0, half2 c1, half2 c2,
//          float norm}: one dwordx4 load fetches a whole site.
// ---------------------------------------------------------------------------
inline size_t field_bytes(const Geom &g, int prec, int nrhs) {
    const int fp = field_prec_of(prec);
    size_t per = fp == HISQ_FP64 ? 48 : fp == HISQ_FP32 ? 24 : 16;
    const int cols = fp == HISQ_FP32 && nrhs >= 2 ? (nrhs + 1) & ~1 : nrhs;
    return (size_t)cols * (size_t)g.vh * per;
}

// ---------------------------------------------------------------------------
// Complex helpers (real arithmetic, written out for the compiler).
// ---------------------------------------------------------------------------
template <typename T> struct cplx {
    T re, im;
};

template <typename T> __device__ __forceinline__ void cmac(cplx<T> &acc, T ar, T ai, cplx<T> b) {
    acc.re = fma(ar, b.re, acc.re);
    acc.re = fma(-ai, b.im, acc.re);
    acc.im = fma(ar, b.im, acc.im);
    acc.im = fma(ai, b.re, acc.im);
}

// acc += conj(a) * b
template <typename T> __device__ __forceinline__ void cmac_conj(cplx<T> &acc, T ar, T ai, cplx<T> b) {
    acc.re = fma(ar, b.re, acc.re);
    acc.re = fma(ai, b.im, acc.re);
    acc.im = fma(ar, b.im, acc.im);
    acc.im = fma(-ai, b.re, acc.im);
}

// Wavefront-wide sum (wave64) by butterfly shuffles.
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace hisq
