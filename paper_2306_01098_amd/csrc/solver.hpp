// Device-resident solver state and the vector kernels of the CG family.
//
// All scalars of the Krylov recurrences (rho, <p,Ap>, alpha, beta, the
// multi-shift zeta's) live in device memory in FP64 and are updated by a
// one-block finalize kernel after each reduction, so an iteration needs no host
// round trip; the host reads the state only once per chunk of iterations.
#pragma once

#include "common.hpp"
#include "access.hpp"

namespace hisq {

// Reliable-update threshold of the mixed-precision solvers: r is replaced by
// the FP64 true residual once the iterated residual has fallen by this factor
// since the last replacement.  Each replacement costs two FP64 operator
// launches; 0.1 (one per decade) -> 0.03 cut the replacements of the 32^3x8
// solves to 1e-10 from 9 to 6 with unchanged iteration counts in every link
// format (FP16N links 8.1 -> 7.6 ms); at 0.01 the FP16N solve needed two more
// iterations.
constexpr double RELIABLE_DELTA = 0.03;

enum {
    FLAG_RUN = 0,       // iterating
    FLAG_CONV = 1,      // iterated residual met the target: check the true residual
    FLAG_BREAKDOWN = 2, // <p, A p> not positive or not finite
    FLAG_RELIABLE = 3,  // reliable update requested (residual fell by delta)
    FLAG_MAXIT = 4,     // iteration limit reached
    FLAG_DONE = 5       // true residual met the target
};

// Per right-hand side (or per shift for the multi-shift solver's base system).
struct alignas(16) CgScalars {
    double rho;      // <r, r> (iterated residual)
    double pq;       // Re <p, A p>
    double beta;     // for p = r + beta p
    double rmax2;    // max <r, r> since the last reliable update
    double target2;  // (tol ||b||)^2
    double delta2;   // reliable-update threshold delta^2 (0: only at convergence)
    double rho_new;  // <r, r> after the last update (kept when a flag is raised)
    double rtrue2;   // ||b - A x||^2 (FP64) at the last true-residual check
    double spare;    // the batch solver's stop time stamp
    double alpha;    // single-reduction CG: the step length of the last update
    int active;      // 1 while the recurrence runs
    int flag;        // FLAG_*
    int iters;       // iterations performed
    int max_iter;
    int nrel;        // reliable updates (residual replacements) so far
    // two-reduction CG: 1 right after a replacement, until p = r + beta p is
    // redone; single-reduction CG: 1 while the next step starts the
    // directions afresh (p = r, s = w)
    int restart;
    int go;          // single-reduction CG: the update kernel steps this column now
    int pad;
};

// Per shift k of the multi-shift solver (Jegerlehner's recurrences, FP64).
struct alignas(16) ShiftScalars {
    double s;         // sigma_k - sigma_0
    double zeta, zeta_old, zeta_new;
    double alpha, beta;
    double target2;   // (tol_k ||b||)^2
    double spare;
    int active;
    int flag;
    int iters;
    int pad;
};

struct MsGlobal {
    double alpha_old, beta_old;
    int nshift;
    int pad;
};

constexpr int MAX_SHIFTS = 32;

// Kernel arguments of the CG vector updates.
struct CgVecParams {
    int vh;
    int nrhs;
    void *x[HISQ_MAX_RHS];  // FP64 solution of each right-hand side (one column each)
    void *r;            // sloppy residual [nrhs]
    void *p;            // sloppy direction [nrhs]
    const void *q;      // sloppy A p [nrhs]
    CgScalars *st;      // [nrhs]
    double *partials;   // [nrhs][gridDim.x]
    // Re <p, A p> block partials of the D_eo kernel, [nrhs][pq_nblk]: summed
    // by every cg_xr_kernel block and again by cg_finalize_kernel, in one
    // fixed order, so no separate reduction launch sits between them
    const double *pq_part;
    int pq_nblk;
    int *skip;          // 1 when no right-hand side is active
    // [nrhs]: 0 while column j waits for its FP64 true residual (set by the
    // finalize kernel with FLAG_CONV / FLAG_RELIABLE, cleared by the
    // true-residual check), else 1; the check's kernels of column j skip on it
    int *tr_skip;
    int *nopend;  // optional: 0 while any column waits for its true residual, else 1
    // multi-shift (nshift > 0): per-shift solutions and directions
    int nshift;
    ShiftScalars *sh;
    MsGlobal *ms;
    void *xs[MAX_SHIFTS];  // FP64 x_k
    void *ps;              // sloppy p_k, [nshift] fields
    // single-reduction CG (r, p as above; q unused):
    void *s;               // sloppy s = A p [nrhs]
    const void *w;         // sloppy w = A r [nrhs] (the D_eo kernel's output)
    // [nrhs][rr_nblk] block partials of <r, r>, Re <r, s> and Re <p, s> of
    // the vectors the update kernel wrote; with the fused step two sets
    // alternate, part_buf doubles apart (0: one set)
    double *rr_part;
    double *rs_part;
    double *ps_part;
    int rr_nblk;
    size_t part_buf;
    const double *rw_part; // [nrhs][rw_nblk] block partials of Re <r, w> (D_eo kernel)
    int rw_nblk;
};

}  // namespace hisq
