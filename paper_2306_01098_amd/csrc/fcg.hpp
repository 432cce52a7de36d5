// Flexible CG with the PTC preconditioner: device state and kernels.
#pragma once

#include "common.hpp"
#include "access.hpp"
#include "solver.hpp"

namespace hisq {

struct alignas(16) FcgScalars {
    double pq;       // Re <p, A p> (written by the Dslash dot epilogue)
    double rtrue2;   // ||b - A x||^2 (FP64) at the last true-residual check
    double2 pr;      // <p, r>
    double2 qz;      // <A p, z>
    double rho;      // ||r||^2 (iterated)
    double rmax2;
    double target2;
    double delta2;
    int active, flag, iters, max_iter;
    int nrel;        // residual replacements
    int pad[3];
};

// Launch flags (ints in device memory): FCG_SKIP while the recurrence is
// stopped, FCG_NOPEND while no true residual is pending, FCG_NORESTART unless
// the last check replaced the residual.
enum { FCG_SKIP = 0, FCG_NOPEND = 1, FCG_NORESTART = 2 };

// skip (nullable): the launches do nothing while *skip != 0.
hipError_t launch_fcg_dot(int vh, const void *a, const void *b, double *partials, double2 *out, hipStream_t st,
                          const int *skip = nullptr);
hipError_t launch_fcg_xr(int vh, void *x, const void *p, const void *q, void *r, FcgScalars *s, double *partials,
                         int *flags, hipStream_t st);
hipError_t launch_fcg_restart(int vh, FcgScalars *s, const double *trpart, int *flags, hipStream_t st);
hipError_t launch_fcg_p(int vh, const void *z, void *p, const FcgScalars *s, hipStream_t st,
                        const int *skip = nullptr);

}  // namespace hisq
