// Host-side declarations shared by the translation units of the library.
#pragma once

#include "common.hpp"
#include "access.hpp"

namespace hisq {

// Compressed formats (reconstruct-12, W14) check every link and synchronize
// st to report in *bad (nullable) whether any link does not fit the format.
hipError_t launch_pack_links(const Geom &g, int prec, const void *fat, const void *naik, void *packed,
                             hipStream_t st, int *bad);
hipError_t launch_unpack_links(const Geom &g, int prec, const void *packed, void *fat, void *naik,
                               hipStream_t st);
hipError_t launch_pack_field(const Geom &g, int prec, int nrhs, const void *src, void *dst, hipStream_t st);
hipError_t launch_unpack_field(const Geom &g, int prec, int nrhs, const void *src, void *dst, hipStream_t st);

// Launch shape of the Dslash: thread mapping (VAR_SITE / VAR_DIR),
// right-hand sides per thread, block size, XCD-aware block order.
struct DslashShape {
    int variant;
    int nin;
    int block;
    int xcd_remap;
};

struct DslashParams;
// lp: link precision; fp: field precision (equal to lp except the mixed
// variant lp = FP16N, fp = FP32).  epi: EPI_PLAIN or EPI_AXPY.
hipError_t launch_dslash(const DslashParams &prm, int lp, int fp, int epi, DslashShape shape,
                         hipStream_t st);
bool dslash_shape_supported(DslashShape s);
// Block order 2 (XCDs take z-slabs) needs N_z divisible by 8; the LDS-staged
// variant also N_y divisible by 8 and 4 N_x in {64, 128, 192, 256}, and (with
// the field precision fp) FP64 or FP32 fields within 64 KiB of staging.
bool dslash_shape_fits(DslashShape s, const Geom &g);
bool dslash_shape_fits(DslashShape s, const Geom &g, int fp);
// Blocks per right-hand side of a Dslash launch in shape s (the number of
// EPI_AXPY_DOT partials per right-hand side).
int dslash_partial_blocks(const Geom &g, DslashShape s);

}  // namespace hisq

namespace hisq {

struct CgVecParams;
int blas_blocks(int vh);
// Block size and count of the single-reduction CG vector kernels (and of
// launch_residual_cols, whose <r, r> partials they share).
int cg_vec_block(int vh);
int cg_vec_blocks(int vh);
hipError_t launch_cg_xr(const CgVecParams &p, int fp, hipStream_t st);
hipError_t launch_cg_p(const CgVecParams &p, int fp, int rhs0, int nrhs, hipStream_t st, bool restart_only = false);
// The true-residual check after r = b - A x of the waiting columns (partials
// in trpart, blas_blocks(vh) per column).
hipError_t launch_cg_restart(const CgVecParams &p, const double *trpart, hipStream_t st);
// Single-reduction CG: the per-column scalar step (after_check: decide the
// columns whose FP64 true residual the check block just formed) and the
// fused vector update with the <r, r> partials of the new residual.
hipError_t launch_cgcg_step(const CgVecParams &p, int fp, int after_check, hipStream_t st);
// r_j = b_j - ax_j for the ncol columns j of packed fields b, ax (FP64)
// whose tr_skip[j] is 0 (every column if tr_skip is NULL), stored in the
// sloppy precision as column col0 + j of the nf-column field r, with the
// block partials of ||r_j||^2 at partials + j * cg_vec_blocks(vh) and, if s
// and p (sloppy nf-column fields like r) are not NULL, those of
// Re <r_j, s_j> and Re <p_j, s_j> at spart / ppart + j * cg_vec_blocks(vh);
// a launch that forms residuals clears *skip and col_off[j] of each column
// it forms (both nullable).
hipError_t launch_residual_cols(int vh, int ncol, int nf, int col0, int fp, const void *b, const void *ax, void *r,
                                double *partials, const int *tr_skip, const void *s, const void *p, double *spart,
                                double *ppart, int *skip, int *col_off, hipStream_t st);
// The scalar and vector steps of single-reduction CG in one launch (every
// block sums its column's partials): state read from st_in, written to
// st_out, partials read from set in_buf and written to the other;
// col_off[j] = 1 while column j is inactive.
struct CgScalars;
hipError_t launch_cgcg_fused(const CgVecParams &p, int fp, const CgScalars *st_in, CgScalars *st_out, int *col_off,
                             int after_check, int in_buf, hipStream_t st);
// r = b - ax (sloppy r) and the block partials of ||b - ax||^2, without the
// sum; the launch does nothing while skip (nullable) points to a nonzero value.
hipError_t launch_residual_parts(int vh, int fp, const void *b, const void *ax, void *r, double *partials,
                                 const int *skip, hipStream_t st);
hipError_t launch_residual(int vh, int fp, const void *b, const void *ax, void *r, double *partials,
                           double *out2, hipStream_t st);
hipError_t launch_norm2(int vh, const void *v, double *partials, double *out2, hipStream_t st);
// out[r] = Re <a_r, b_r> for n FP64 fields (partials: n * blas_blocks(vh) doubles).
hipError_t launch_dot_re(int vh, int n, const void *a, const void *b, double *partials, double *out, hipStream_t st);
// dst = src for n16 16-byte chunks (non-temporal streaming copy).
hipError_t launch_stream_copy(const void *src, void *dst, size_t n16, hipStream_t st);
// Blocks of the read reference for n16 chunks of 16 bytes (= sink words).
size_t stream_read_blocks(size_t n16);
hipError_t launch_stream_read(const void *src, size_t n16, unsigned *sink, hipStream_t st);
// out[s * stride] = sum over nblk block partials of slot s (one-block kernel);
// does nothing when skip is non-NULL and *skip != 0.
hipError_t launch_sum_partials(const double *partials, int nslots, int nblk, double *out, int stride,
                               const int *skip, hipStream_t st);
hipError_t launch_copy(int vh, int n, int fs, int fd, const void *src, void *dst, hipStream_t st);
// dst (a one-column field) = column k of the n-column field src (FP64 or FP32).
hipError_t launch_copy_col(int vh, int fp, int n, int k, const void *src, void *dst, hipStream_t st);
hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t st);

}  // namespace hisq
