/*
 * hisq.h -- C ABI of the MI355X (gfx950) HISQ staggered Dslash / CG library.
 *
 * The operator is the HISQ Dslash of the paper's Sec. 5.1 ("HISQ Dslash
 * performance model", the stencil equation there):
 *
 *   (D psi)(x) = sum_mu eta_mu(x) [ X_mu(x) psi(x+mu)  - X_mu(x-mu)^+  psi(x-mu)
 *                                 + W_mu(x) psi(x+3mu) - W_mu(x-3mu)^+ psi(x-3mu) ]
 *
 * with X the fat (smeared) links, W the long three-hop links, the
 * Kogut-Susskind phases eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y),
 * eta_3 = (-1)^(x+y+z), periodic links and colour vectors periodic in space and
 * periodic or antiperiodic in time (Sec. 3, "Physics modules").  Coefficients
 * (c_1, c_Naik, ...) are folded into X and W by the caller; the phases and the
 * time boundary sign are applied by the library, never folded into the links.
 * D_eo maps odd sites to even sites and D_oe even to odd (the first index is
 * the output parity); the solvers work with the even-site normal operator
 * M_e = m^2 - D_eo D_oe, the role of the applyMdaggM operator of Sec. 3.2
 * ("Inverters").
 *
 * Conventions for every entry point:
 *  - Every buffer argument is device memory owned by the caller (for example
 *    a torch tensor on the GPU) unless its comment says "host".  The library
 *    never allocates or frees caller-visible memory.  Sizes of packed buffers
 *    and workspaces come only from the *_bytes queries below.
 *  - Canonical layouts (complex128, interleaved re/im):
 *      links  (4, Nt, Nz, Ny, Nx, 3, 3): [mu][t][z][y][x][row][col], x fastest;
 *      fields (nrhs, V/2, 3): the sites of one parity in increasing
 *             lexicographic order lex = x + Nx (y + Ny (z + Nz t)), i.e. the
 *             half-lattice index floor(lex/2) of the even/odd memory order of
 *             Sec. 4.3 ("Indexing and fields").
 *    Packed layouts are private to the library (structure of arrays split by
 *    parity, direction and matrix chunk); convert with the pack/unpack calls.
 *    A packed field of n columns is one buffer of hisq_field_bytes(lat, prec,
 *    n) bytes.  For HISQ_FP64 and HISQ_FP16N it is the n one-column fields
 *    one after another; HISQ_FP32 fields of two or more columns interleave
 *    the columns in pairs (one 16-byte record per site, colour and pair; for
 *    odd n the last pair has an unused slot, so the field takes the bytes of
 *    n + 1 columns), and a column of such a field is not a one-column field
 *    at an offset.
 *  - Every call returns a hisq_status.  Nothing throws, aborts or exits across
 *    the ABI.  Arguments are validated on the host before any HIP call;
 *    hisq_last_error() returns a message for the calling thread's last error.
 *  - pack, unpack, dslash and apply_m are asynchronous on `stream` (a
 *    hipStream_t; NULL is the default stream).  The solvers are synchronous:
 *    they return when finished because they report convergence.
 *  - Calls are re-entrant given distinct output and workspace buffers.
 */
#ifndef HISQ_H
#define HISQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Lattice descriptor.  dims = {Nx, Ny, Nz, Nt}; each extent even and >= 4 so
 * that parity is consistent across the periodic wrap and floor(lex/2) is a
 * bijection on each parity.  t_bc = +1 (periodic) or -1 (antiperiodic) time
 * boundary condition of the colour vectors. */
typedef struct {
    int32_t dims[4];
    int32_t t_bc;
} hisq_lattice;

/* Storage precision of packed links and fields.
 *   HISQ_FP64  : binary64, arithmetic in FP64.
 *   HISQ_FP32  : binary32, arithmetic in FP32.
 *   HISQ_FP16N : links in binary16 (each part rounded once, from binary64,
 *                to nearest-even binary16); colour vectors in binary16 scaled
 *                by a binary32 per-site norm n = max |component| over the 6
 *                reals of the site (packing from complex128: each part v is
 *                stored as binary16(v / binary32(n)), quotient in FP64 rounded
 *                once); arithmetic in FP32.
 *   HISQ_FP64R12, HISQ_FP32R12 : compressed links for special-unitary link
 *                fields (the gauge-field compression types of Sec. 4.4, whose
 *                missing entries follow from the SU(3) symmetry, Sec. 5): only
 *                rows 0 and 1 of each matrix are stored (12 reals, rounded as
 *                for HISQ_FP64 / HISQ_FP32); row 2 is rebuilt in-kernel as the
 *                complex conjugate of the cross product of rows 0 and 1, which
 *                is exact for SU(3) and wrong for anything else.
 *                hisq_pack_links checks every link (X and W) and refuses
 *                (HISQ_ERR_INVALID_ARG) links whose rebuilt row 2 differs from
 *                the given one by more than 1e-10 (FP64R12) or 1e-5 (FP32R12)
 *                times the matrix's Frobenius norm: HISQ fat links, and the
 *                U(3) Naik links of hisq_smear_links, are refused.
 *   HISQ_FP64W14, HISQ_FP32W14 : fat links X stored in full (as HISQ_FP64 /
 *                HISQ_FP32); Naik links W stored as rows 0 and 1 plus one
 *                complex factor z (14 reals), row 2 rebuilt in-kernel as
 *                z conj(row 0 x row 1).  z = <c, row 2> / <c, c> with
 *                c = conj(row 0 x row 1) is formed from the FP64 input; the
 *                form is exact for SU(3) (z = 1), U(3) (z = det) and real
 *                multiples a V of U(3) matrices (z = det V / a), such as the
 *                HISQ Naik link c_Naik Y(x) Y(x+mu) Y(x+2mu) with Y in U(3)
 *                that hisq_smear_links returns.  hisq_pack_links refuses
 *                (HISQ_ERR_INVALID_ARG) Naik links that the form does not
 *                reproduce to 1e-10 (FP64W14) or 1e-5 (FP32W14) of their
 *                Frobenius norm.  Bytes per Dslash output site: 2144 (FP64W14)
 *                and 1072 (FP32W14), against 2400 and 1200 uncompressed.
 *                Reconstruct-12 and W14 packing synchronize `stream` (they
 *                read the check's result back) and are serialized within the
 *                process.  Colour vectors and arithmetic of the R12 and W14
 *                formats are those of HISQ_FP64 / HISQ_FP32, so their fields
 *                are HISQ_FP64 / HISQ_FP32 fields.  Accepted by the
 *                pack/unpack calls, hisq_dslash, hisq_apply_m (and _dot), the
 *                autotuner, and as the `inner` precision of hisq_cg and
 *                hisq_multishift_cg (links_inner in this format). */
typedef enum {
    HISQ_FP64 = 0,
    HISQ_FP32 = 1,
    HISQ_FP16N = 2,
    HISQ_FP64R12 = 3,
    HISQ_FP32R12 = 4,
    HISQ_FP64W14 = 5,
    HISQ_FP32W14 = 6
} hisq_prec;

typedef enum {
    HISQ_OK = 0,
    HISQ_ERR_INVALID_ARG = 1,
    HISQ_ERR_NOT_CONVERGED = 2,
    HISQ_ERR_BREAKDOWN = 3,
    HISQ_ERR_DEVICE = 4,
    HISQ_ERR_WORKSPACE = 5,
    HISQ_ERR_UNSUPPORTED = 6
} hisq_status;

/* Per-solve report (host).  true_residual = ||b - A x|| / ||b|| recomputed
 * in FP64 with FP64 links at the end of the solve; reliable_updates = how
 * often the iterated residual was replaced by the FP64 b - A x and the
 * recurrence restarted from it (reliable updates, and convergence signals the
 * true residual did not confirm); seconds = wall time of the call.
 * Multi-shift solves split `iterations` into shared_iterations (iterations of
 * the shared Krylov space until this shift was frozen) and
 * refine_iterations (iterations of this shift's refinement CG afterwards);
 * every other solver reports shared_iterations = refine_iterations = 0. */
typedef struct {
    int32_t iterations;
    int32_t reliable_updates;
    double true_residual;
    double seconds;
    int32_t shared_iterations;
    int32_t refine_iterations;
} hisq_solve_info;

/* Opaque context: device ordinal and the autotuning cache.  May be NULL in
 * every call, meaning the current device and built-in launch shapes. */
typedef struct hisq_context hisq_context;

hisq_status hisq_context_create(hisq_context **ctx, int32_t device);
void hisq_context_destroy(hisq_context *ctx);
const char *hisq_status_string(hisq_status s);
/* Message describing the calling thread's most recent error ("" if none). */
const char *hisq_last_error(void);

/* Maximum number of right-hand sides per call. */
#define HISQ_MAX_RHS 16

/* Bytes of the packed X and W links of one lattice (both parities). */
size_t hisq_links_bytes(const hisq_lattice *lat, hisq_prec prec);
/* Bytes of a packed colour-vector field of nrhs columns on one parity (V/2
 * sites; HISQ_FP32 with odd nrhs >= 3: nrhs + 1 columns, see the layouts above). */
size_t hisq_field_bytes(const hisq_lattice *lat, hisq_prec prec, int32_t nrhs);

/* Pack canonical complex128 links fat_c128 (X) and naik_c128 (W), each of
 * 4*V*9 complex, into `packed` (hisq_links_bytes).  Asynchronous. */
hisq_status hisq_pack_links(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec,
                            const void *fat_c128, const void *naik_c128, void *packed,
                            void *stream);
/* Inverse of hisq_pack_links: widen packed links back to canonical complex128
 * fat_c128 / naik_c128 (each 4*V*9 complex).  Asynchronous. */
hisq_status hisq_unpack_links(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec,
                              const void *packed, void *fat_c128, void *naik_c128, void *stream);
/* Pack nrhs canonical half-lattice fields (nrhs*V/2*3 complex128) into
 * `packed` (hisq_field_bytes).  For HISQ_FP16N the per-site norm is formed
 * from the FP64 input as documented at hisq_prec.  Asynchronous. */
hisq_status hisq_pack_field(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec,
                            int32_t nrhs, const void *half_c128, void *packed, void *stream);
/* Inverse of hisq_pack_field (exact widening to complex128). */
hisq_status hisq_unpack_field(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec,
                              int32_t nrhs, const void *packed, void *half_c128, void *stream);

/* out = D_eo in (out_parity 0: odd input, even output) or D_oe in
 * (out_parity 1), for nrhs packed fields.  links: packed with the same prec.
 * `in` and `out` must not overlap.  Asynchronous.  Paper Sec. 5.1; the
 * multi-RHS form (one link load shared by all right-hand sides) follows the
 * N_inner / N_outer scheme described there. */
hisq_status hisq_dslash(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec,
                        int32_t out_parity, const void *links, const void *in, void *out,
                        int32_t nrhs, void *stream);

/* HISQ link smearing (the two-level treatment of Sec. 3.1): from thin links
 * U, level 1 (1-link 1/8, 3-link staples 1/16, 5-link 1/64, 7-link 1/384)
 * gives V; Y = V (V^+ V)^(-1/2) projects it to U(3); level 2 from Y (1-link
 * 1, 3-link 1/16, 5-link 1/64, 7-link 1/384, Lepage -1/8) gives the fat links
 * X, and W_mu(x) = c_Naik Y_mu(x) Y_mu(x+mu) Y_mu(x+2mu) with
 * c_Naik = -1/24 + naik_eps/8 the Naik links; links periodic.  All three
 * fields are device complex128 arrays in the canonical layout
 * (4, Nt, Nz, Ny, Nx, 3, 3) (pass fat and naik to hisq_pack_links).  FP64.
 *   ws  workspace of hisq_smear_workspace_bytes(lat) bytes (44 matrices per site).
 * thin, fat and naik must be distinct.  Asynchronous. */
size_t hisq_smear_workspace_bytes(const hisq_lattice *lat);
hisq_status hisq_smear_links(hisq_context *ctx, const hisq_lattice *lat, const void *thin_c128, double naik_eps,
                             void *fat_c128, void *naik_c128, void *ws, size_t ws_bytes, void *stream);

/* Bandwidth reference for the roofline: dst = src for `bytes` bytes with the
 * library's streaming copy kernel (16-byte loads and stores, four per
 * thread, non-temporal).  bytes must be a positive multiple of 16 and both
 * pointers 16-byte aligned device memory that does not overlap; otherwise
 * HISQ_ERR_INVALID_ARG.  Asynchronous.  Not part of the method: it measures
 * the copy ceiling the Dslash rates are compared with. */
hisq_status hisq_stream_copy(hisq_context *ctx, const void *src, void *dst, size_t bytes, void *stream);

/* Read-only bandwidth reference: reads `bytes` bytes of src (16-byte
 * non-temporal loads, four per thread, blocks of 1024 chunks) and stores in
 * sink[b] the XOR of the 32-bit words of block b's 16 KiB (the last block:
 * what remains).  sink: device array of hisq_stream_read_sink_words(bytes)
 * uint32 (0 when bytes is not a multiple of 16), 4-byte aligned, not
 * overlapping src.  bytes a positive multiple of 16, src 16-byte aligned;
 * otherwise HISQ_ERR_INVALID_ARG.  Asynchronous.  Not part of the method: the
 * Dslash reads 98 % of its bytes, so this is the ceiling its rate is compared
 * with, next to the copy. */
size_t hisq_stream_read_sink_words(size_t bytes);
hisq_status hisq_stream_read(hisq_context *ctx, const void *src, size_t bytes, uint32_t *sink, void *stream);

/* out_even = (m^2) in_even - D_eo D_oe in_even, using tmp_odd (a packed
 * field of nrhs on the odd sites) as scratch.  Asynchronous. */
hisq_status hisq_apply_m(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec,
                         double mass, const void *links, const void *in_even, void *out_even,
                         void *tmp_odd, int32_t nrhs, void *stream);

/* out_even = (m^2) in_even - D_eo D_oe in_even as in hisq_apply_m, with the
 * link and field precisions given separately so that every operator the
 * solvers iterate with can be applied on its own, and
 * dot_out[r] = Re <in_r, out_r> for each right-hand side r: the fused
 * <p, M_e p> of the CG iteration (Sec. 3.2), summed in FP64 over the
 * products of the loaded in-values and the computed out-values before the
 * out field is rounded to its storage format, block partials first and then
 * one fixed-order pass (deterministic).
 *   link_prec, field_prec  one of the pairs the solvers use: (FP64, FP64),
 *               (FP32, FP32), (FP16N, FP16N), (FP16N, FP32) (binary16 links
 *               with FP32 vectors, the inner operator of hisq_cg with
 *               inner = HISQ_FP16N), (FP64R12, FP64), (FP32R12, FP32),
 *               (FP64W14, FP64), (FP32W14, FP32);
 *               anything else is HISQ_ERR_INVALID_ARG.
 *   links       packed links of link_prec; in_even, out_even (even sites) and
 *               tmp_odd (odd sites, scratch) packed fields of nrhs columns in
 *               field_prec; distinct buffers.
 *   dot_out     device array of nrhs doubles.
 *   ws          device workspace of hisq_apply_m_dot_workspace_bytes(lat, nrhs)
 *               bytes (the block partials).
 * The launch shape is the one hisq_get_dslash_shape reports for link_prec
 * (a shape set for HISQ_FP16N covers both FP16N pairs).  Asynchronous. */
size_t hisq_apply_m_dot_workspace_bytes(const hisq_lattice *lat, int32_t nrhs);
hisq_status hisq_apply_m_dot(hisq_context *ctx, const hisq_lattice *lat, hisq_prec link_prec,
                             hisq_prec field_prec, double mass, const void *links, const void *in_even,
                             void *out_even, void *tmp_odd, int32_t nrhs, double *dot_out, void *ws,
                             size_t ws_bytes, void *stream);

/* Bytes of the device scratch array behind hisq_apply_m_dot_noalloc (per
 * device that runs it, held until the process ends). */
#define HISQ_NOALLOC_SCRATCH_BYTES (4u << 20)

/* hisq_apply_m_dot without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the block partials live in a file-scope
 * device array of HISQ_NOALLOC_SCRATCH_BYTES bytes, one per device, whose
 * address the library looks up once per device (at hisq_context_create, or
 * at the first call on a device).  The call allocates nothing: no hipMalloc,
 * hipFree or allocating library routine.  Same arguments, operators, launch
 * shape and results as hisq_apply_m_dot (bitwise: the same kernels).
 * Limit: the call needs nrhs * (block count of the launch shape) doubles of
 * partials; every call with hisq_apply_m_dot_workspace_bytes(lat, nrhs) <=
 * HISQ_NOALLOC_SCRATCH_BYTES fits (e.g. 32^4 with 4 rhs, or 48^3x12 with 3);
 * larger calls fit when their launch shape has enough sites per block (the
 * built-in shapes of 32^4 and 48^3x12 with 16 rhs do); a call whose shape
 * needs more returns HISQ_ERR_WORKSPACE before any launch.  Every call
 * on one device shares that device's array: each call writes every partial
 * it reads, but calls that overlap in time on one device (concurrent streams
 * or threads) race and give wrong dot products.  Asynchronous. */
hisq_status hisq_apply_m_dot_noalloc(hisq_context *ctx, const hisq_lattice *lat, hisq_prec link_prec,
                                     hisq_prec field_prec, double mass, const void *links, const void *in_even,
                                     void *out_even, void *tmp_odd, int32_t nrhs, double *dot_out, void *stream);

/* Workspace bytes for hisq_cg (nshift = 0) or hisq_multishift_cg (nrhs = 1,
 * nshift shifts) with inner precision `inner`.  0 on invalid arguments. */
size_t hisq_cg_workspace_bytes(const hisq_lattice *lat, hisq_prec inner, int32_t nrhs, int32_t nshift);

/* Solve (m^2 - D_eo D_oe) x_k = b_k for nrhs independent right-hand sides
 * (the CG of Sec. 3.2, "Inverters", with its multi-right-hand-side form: the
 * columns share every Dslash launch and link load but keep their own Krylov
 * scalars; a converged column stops updating).
 *   links_f64   packed HISQ_FP64 links (always required: the true residual
 *               b - A x is formed in FP64 with them).
 *   links_inner packed links of precision `inner` for the iterations, or NULL
 *               when inner == HISQ_FP64.  With inner = HISQ_FP32 or FP16N the
 *               iteration vectors are FP32 and the solver is reliable-update
 *               mixed-precision CG: x is accumulated in FP64, all inner
 *               products and norms are FP64, and r is replaced by the FP64
 *               b - A x whenever the iterated residual falls below 0.03
 *               times its largest value since the last replacement.
 *   b, x        packed HISQ_FP64 fields of nrhs columns on the even sites;
 *               x holds the initial guess on entry and the solution on exit.
 *   tol         stop when ||b - A x|| <= tol ||b|| (FP64 true residual).
 *   ws          workspace of hisq_cg_workspace_bytes(lat, inner, nrhs, 0).
 *   info        host array [nrhs], filled on every return after argument checks.
 * Returns HISQ_ERR_NOT_CONVERGED after max_iter iterations (x holds the last
 * iterate), HISQ_ERR_BREAKDOWN on <p, A p> <= 0 or non-finite values.
 * Synchronous: returns when done. */
hisq_status hisq_cg(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                    const void *links_inner, hisq_prec inner, int32_t nrhs, const void *b, void *x, double tol,
                    int32_t max_iter, void *ws, size_t ws_bytes, hisq_solve_info *info, void *stream);

/* Stochastic chiral condensate (an observable of Sec. 3.3, measured there with
 * a small number of random vectors):
 *   pbp = (1/V) Tr (D + m)^-1 = (2 m / V) Tr_e M_e^-1,
 * (the odd-site block has the spectrum of M_e and D (m^2 - D^2)^-1 is
 * traceless), estimated as the mean of s_i = (2 m / V) Re <eta_i, M_e^-1 eta_i>
 * over nnoise caller-drawn noise vectors with E[eta eta^+] = 1 (e.g. complex
 * Gaussian with E|eta_k|^2 = 1).  The solves run as multi-RHS hisq_cg in
 * groups of up to HISQ_MAX_RHS; the dot products are FP64 reductions on the
 * device.
 *   noise    packed HISQ_FP64 even fields [nnoise]
 *   x        packed HISQ_FP64 even fields [nnoise] (overwritten with
 *            M_e^-1 eta_i; initial guess zero); must not alias noise
 *   samples  host array [nnoise] or NULL: the s_i
 *   pbp      host pointer: the mean; err host pointer or NULL: its standard
 *            error (NaN for nnoise = 1)
 *   ws       workspace of hisq_cg_workspace_bytes(lat, inner, min(nnoise, 16), 0)
 *   info     host array [nnoise] or NULL
 * Other arguments and statuses as for hisq_cg (the worst status of the
 * groups).  Synchronous. */
hisq_status hisq_chiral_condensate(hisq_context *ctx, const hisq_lattice *lat, double mass,
                                   const void *links_f64, const void *links_inner, hisq_prec inner,
                                   int32_t nnoise, const void *noise, void *x, double tol, int32_t max_iter,
                                   void *ws, size_t ws_bytes, double *samples, double *pbp, double *err,
                                   hisq_solve_info *info, void *stream);

/* Multi-shift CG (Sec. 3.2): solve (m^2 - D_eo D_oe + shifts[k]) x[k] = b for
 * nshift (1..32) shifts at the cost of one operator application per iteration:
 * the Krylov space of the smallest shift is built and the other shifts follow
 * Jegerlehner's recurrences (zeta, alpha_k, beta_k in FP64); a shift is frozen
 * once |zeta_k| ||r|| <= tol[k] ||b||.  Afterwards every shift whose FP64 true
 * residual is above tol[k] is refined by (reliable-update) CG from x[k].
 *   shifts, tol  host arrays [nshift]; m^2 + shifts[k] > 0.
 *   x            host array of nshift distinct device pointers to packed
 *                HISQ_FP64 fields (overwritten; the initial guess is zero).
 *   ws           workspace of hisq_cg_workspace_bytes(lat, inner, 1, nshift).
 *   info         host array [nshift]; iterations = shared Krylov iterations up
 *                to the freeze (shared_iterations) + refinement iterations
 *                (refine_iterations).
 * Other arguments and statuses as for hisq_cg.  Synchronous. */
hisq_status hisq_multishift_cg(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                               const void *links_inner, hisq_prec inner, int32_t nshift, const double *shifts,
                               const void *b, void *const *x, const double *tol, int32_t max_iter, void *ws,
                               size_t ws_bytes, hisq_solve_info *info, void *stream);

/* The shared Krylov phase of hisq_multishift_cg alone, without the
 * refinement: on return x[k] holds the multi-shift iterate of shift k at the
 * iteration where it was frozen (|zeta_k| ||r|| <= tol[k] ||b||, or where the
 * smallest shift met its own tolerance), info[k].iterations =
 * info[k].shared_iterations = that iteration, and info[k].true_residual its
 * FP64 true residual ||b - (M_e + shifts[k]) x[k]|| / ||b||.  Returns HISQ_OK
 * when every shift meets its tolerance, HISQ_ERR_NOT_CONVERGED otherwise
 * (with a reduced-precision inner operator the Krylov iterates stall near
 * that precision, which is why hisq_multishift_cg refines them).  Same
 * arguments and workspace as hisq_multishift_cg.  Synchronous. */
hisq_status hisq_multishift_krylov(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                                   const void *links_inner, hisq_prec inner, int32_t nshift, const double *shifts,
                                   const void *b, void *const *x, const double *tol, int32_t max_iter, void *ws,
                                   size_t ws_bytes, hisq_solve_info *info, void *stream);

/* One problem of a batched solve. */
typedef struct {
    hisq_lattice lat;
    double mass;
    const void *links_f64;   /* packed HISQ_FP64 links of this lattice */
    const void *links_inner; /* packed links of the batch's inner precision (NULL for FP64) */
    const void *b;           /* packed HISQ_FP64 field, even sites */
    void *x;                 /* packed HISQ_FP64 field: initial guess in, solution out */
    double tol;              /* ||b - M_e x|| <= tol ||b|| */
} hisq_problem;

/* Workspace bytes of hisq_cg_batch for these problems (0 on invalid input). */
size_t hisq_cg_batch_workspace_bytes(int32_t nproblems, const hisq_problem *problems, hisq_prec inner);

/* Batched CG: nproblems (1..256) independent systems M_e x = b, each on its
 * own lattice with its own mass, links and tolerance, solved together.  Every
 * launch covers the sites of all problems through a block -> problem work
 * list (its sites per block, 64, 128 or 256, chosen per call by timing one
 * batch-wide Dslash launch of each), so one iteration of all problems is four
 * kernels (plus the finalize kernels of the two reductions); chunks of
 * iterations are captured in a HIP graph and replayed; a problem whose
 * iterated residual meets its target stops updating while the others go on.
 * With inner = FP32/FP16N the iterations use that link precision with FP32
 * vectors and FP64 reliable updates (batched over the problems that need
 * one), as in hisq_cg.  The compressed (R12, W14) precisions are not accepted here
 * (HISQ_ERR_UNSUPPORTED; the workspace query returns 0).
 *   problems    host array [nproblems]; the structs may be freed on return.
 *   info        host array [nproblems] (seconds = wall time of the batch).
 *   latency_s   host array [nproblems] or NULL: device-clock time from the
 *               start of the batched iterations to the FP64 true-residual
 *               check that confirmed the problem's solution.
 * Statuses as for hisq_cg (NOT_CONVERGED / BREAKDOWN if any problem ends so).
 * Synchronous. */
hisq_status hisq_cg_batch(hisq_context *ctx, int32_t nproblems, const hisq_problem *problems, hisq_prec inner,
                          int32_t max_iter, void *ws, size_t ws_bytes, hisq_solve_info *info, double *latency_s,
                          void *stream);

/* ---------------------------------------------------------------------------
 * Learned preconditioner: a parallel-transport convolution (PTC) network.
 * The paper has no such component; the network follows the gauge-equivariant
 * PTC layers of Lehner and Wettig (arXiv:2302.05419):
 *   layer:  out_c(x) = sum_{c'} sum_p w[c][c'][p] (T_p in_{c'})(x),
 *   paths:  p = 0 identity; 1 + 2mu: (T psi)(x) = X_mu(x) psi(x+mu);
 *           2 + 2mu: (T psi)(x) = X_mu(x-mu)^+ psi(x-mu), time-boundary sign
 *           on a hop that wraps (X = the fat links),
 *   network: channels 1 -> 8 -> 8 -> 1, no bias, no nonlinearity, on the
 *           whole lattice; input = an even-site field extended by zero,
 *           output read on the even sites.
 * Weights: HISQ_PTC_NWEIGHTS complex numbers, layer after layer, each layer
 * [c_out][c_in][path]; the kernels read them as FP32 (interleaved float2);
 * training keeps FP64 master weights and Adam moments (double2).
 * Fields here are packed HISQ_FP32 (links: the packed FP32 links of the
 * lattice; only X is used).
 * ------------------------------------------------------------------------- */
#define HISQ_PTC_NWEIGHTS 720

/* Workspace of the network (activations of one application, gradients). */
size_t hisq_ptc_workspace_bytes(const hisq_lattice *lat);
/* out_even = N(in_even).  Keeps the activations in ws for hisq_ptc_backward.
 * Asynchronous. */
hisq_status hisq_ptc_forward(hisq_context *ctx, const hisq_lattice *lat, const void *links_f32, const void *weights,
                             const void *in_even, void *out_even, void *ws, size_t ws_bytes, void *stream);
/* Backward pass of the last hisq_ptc_forward with this ws: given the gradient
 * g_out_even = dL/dRe y + i dL/dIm y of a real loss L, adds dL/dRe w + i dL/dIm w
 * to grad (double2 [HISQ_PTC_NWEIGHTS], FP64 sums over sites in a fixed order)
 * and writes the input gradient to g_in_even if it is not NULL.  Asynchronous. */
hisq_status hisq_ptc_backward(hisq_context *ctx, const hisq_lattice *lat, const void *links_f32,
                              const void *weights, const void *g_out_even, void *g_in_even, void *grad, void *ws,
                              size_t ws_bytes, void *stream);
/* One Adam step (real and imaginary parts as separate parameters; step counts
 * from 1) on FP64 master weights w_master with moments m, v (double2
 * [HISQ_PTC_NWEIGHTS]); also refreshes the FP32 copy w_f32.  Asynchronous. */
hisq_status hisq_ptc_adam_step(hisq_context *ctx, void *w_master, void *w_f32, const void *grad, void *m, void *v,
                               int32_t step, double lr, double beta1, double beta2, double eps, void *stream);
/* One training step on `batch` (source, solution) pairs of M_e x_i = b_i
 * (src_f32: the sources as one packed FP32 field of `batch` columns; sol_f64:
 * the solutions as one packed FP64 field of `batch` columns, e.g. from
 * hisq_cg).  Loss: the error of the network's
 * approximation in the energy norm that CG minimises,
 *   L = (1/B) sum_i <e_i, M_e e_i> / <x_i, b_i>,   e_i = N(b_i) - x_i,
 * with M_e applied in FP32 (mass, FP32 links); gradients by the backward pass
 * of hisq_ptc_backward, then one Adam step.  *loss (host) receives L before
 * the update.  Synchronous. */
hisq_status hisq_ptc_train_step(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f32,
                                void *w_master, void *w_f32, void *m, void *v, int32_t step, int32_t batch,
                                const void *src_f32, const void *sol_f64, double lr, double beta1, double beta2,
                                double eps, double *loss, void *ws, size_t ws_bytes, void *stream);

/* Workspace of hisq_fcg. */
size_t hisq_fcg_workspace_bytes(const hisq_lattice *lat);
/* Flexible CG (Notay, one-vector truncation) for M_e x = b with z = N(r) as
 * the preconditioner: alpha = <p, r> / <p, A p>, p <- z - (<A p, z> / <p, A p>) p.
 * FP32 links and iteration vectors, FP64 x, FP64 inner products; when the
 * iterated residual falls by 10x or meets the target, the FP64 true residual
 * replaces r and the recurrence continues from it.  Stops on the FP64 true
 * residual <= tol ||b||.  b, x: packed HISQ_FP64 even fields; x holds the
 * initial guess.  Statuses as for hisq_cg.  Synchronous. */
hisq_status hisq_fcg(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                     const void *links_f32, const void *weights, const void *b, void *x, double tol,
                     int32_t max_iter, void *ws, size_t ws_bytes, hisq_solve_info *info, void *stream);

/* Launch shape of hisq_dslash (and of the Dslash inside the solvers).
 *   variant   0: one thread per output site; 1: four lanes per site, one per
 *             direction, combined by wavefront shuffles; 2: one thread per
 *             site, a block per piece of 8 y-rows x N_x/2 sites at fixed
 *             (t, z) in the z-slab order, whose x- and y-hop neighbour
 *             vectors are first staged in LDS (block and xcd_remap are then
 *             set by the library: 4 N_x threads, order 2; needs N_z and N_y
 *             divisible by 8, N_x in {16, 32, 48, 64} and FP64 or FP32
 *             fields within 64 KiB of LDS per block, else
 *             hisq_set_dslash_shape returns HISQ_ERR_INVALID_ARG; with FP16N
 *             fields the launch falls back to variant 0); 3: sixteen lanes
 *             per site, lane k computing hop k alone, combined by four
 *             butterfly shuffles (for small lattices; nin 1 or 2).
 *   nin       right-hand sides per thread sharing each link load (1, 2, 4, 8;
 *             the remaining right-hand sides run as further blocks: the
 *             N_inner x N_outer split of the paper's Sec. 5.1; a one-column
 *             HISQ_FP32 field runs with nin 1).
 *   block     threads per block (64, 128, 256).
 *   xcd_remap block order.  0: blocks in site order (dealt round-robin over
 *             the 8 XCDs); 1: each XCD takes one contiguous 1/8 of the sites
 *             (a range in t); 2: each XCD takes one z-slab of N_z / 8 planes
 *             for every t, so only the hops in z cross XCDs (needs N_z
 *             divisible by 8; HISQ_ERR_INVALID_ARG from hisq_set_dslash_shape
 *             otherwise); with several right-hand sides and N_y divisible by
 *             8 the slab is swept in bands of 8 y-rows. */
typedef struct {
    int32_t variant;
    int32_t nin;
    int32_t block;
    int32_t xcd_remap;
} hisq_dslash_shape;

/* Autotuner: time every supported shape of hisq_dslash for (lattice, prec,
 * nrhs) on the caller's buffers (out is overwritten) and keep the fastest in
 * ctx (required).  Synchronous on `stream`. */
hisq_status hisq_tune_dslash(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, int32_t nrhs,
                             const void *links, const void *in, void *out, void *stream);
/* The shape hisq_dslash will use (tuned or set in ctx, else the built-in
 * default; ctx may be NULL).  *shape is a host pointer. */
hisq_status hisq_get_dslash_shape(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, int32_t nrhs,
                                  hisq_dslash_shape *shape);
/* Force a shape for (lattice, prec, nrhs) in ctx (required). */
hisq_status hisq_set_dslash_shape(hisq_context *ctx, const hisq_lattice *lat, hisq_prec prec, int32_t nrhs,
                                  const hisq_dslash_shape *shape);

#ifdef __cplusplus
}
#endif

#endif /* HISQ_H */
