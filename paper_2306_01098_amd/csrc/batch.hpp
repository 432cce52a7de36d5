// Shared definitions of the batched (many independent lattices) CG.
#pragma once

#include "common.hpp"
#include "solver.hpp"

namespace hisq {

// Sites (threads) per block of the batch kernels: 64, 128 or 256, chosen per
// batch by timing one Dslash launch of each (the work list depends on it).
constexpr int BATCH_BLOCK_MIN = 64;
constexpr int MAX_BATCH = 256;    // problems per batch

// One problem of the batch, as the kernels see it.
struct BatchProb {
    Geom g;
    double m2;
    const char *links_in;  // iteration precision
    const char *links64;   // FP64 (true residuals)
    const void *b;         // FP64 source
    void *x;               // FP64 solution
    void *r, *p, *q, *t;   // iteration vectors (sloppy precision); t on odd sites
    void *ax, *t64;        // FP64 scratch: M x (even) and D_oe x (odd)
    int first_blk, nblk;   // this problem's range of the work list
};

struct BatchArgs {
    const BatchProb *probs;
    int nprob;
    const int *blk_prob;  // work list: problem of each block
    CgScalars *st;        // [nprob]
    int *mask;            // [nprob] problems taking part in a true-residual pass
    double *partials;     // [nblocks]
    int *nactive;         // problems still iterating: iteration kernels do nothing at 0
    int *npend;           // nonzero while some problem waits for its true residual
    int block;            // sites per block (64, 128, 256)
};

enum { ROLE_ITER_DOE = 0, ROLE_ITER_DEO = 1, ROLE_TRUE_DOE = 2, ROLE_TRUE_DEO = 3 };
enum {
    BOP_ITER_DOE = 0, BOP_ITER_DEO, BOP_TRUE_DOE, BOP_TRUE_DEO, BOP_XR, BOP_P, BOP_RESIDUAL,
    BOP_RESIDUAL_COPY_P, BOP_BNORM,
    BOP_RESTART  // true-residual decision of the masked problems, then p = r + beta p for the restarted
};

hipError_t launch_batch(const BatchArgs &a, int nblocks, int op, int lp, hipStream_t st);
hipError_t launch_batch_bnorm(const BatchArgs &a, int nblocks, double *bnorm2, hipStream_t st);
hipError_t launch_batch_clock(double *out, hipStream_t st);

}  // namespace hisq
