// Flexible CG with the PTC preconditioner: device state and kernels.
#pragma once

#include "common.hpp"
#include "access.hpp"
#include "solver.hpp"

namespace hisq {

struct alignas(16) FcgScalars {
    double pq;       // Re <p, A p> (written by the Dslash dot epilogue)
    double pad0;
    double2 pr;      // <p, r>
    double2 qz;      // <A p, z>
    double rho;      // ||r||^2 (iterated)
    double rmax2;
    double target2;
    double delta2;
    int active, flag, iters, max_iter;
};

hipError_t launch_fcg_dot(int vh, const void *a, const void *b, double *partials, double2 *out, hipStream_t st);
hipError_t launch_fcg_xr(int vh, void *x, const void *p, const void *q, void *r, FcgScalars *s, double *partials,
                         hipStream_t st);
hipError_t launch_fcg_p(int vh, const void *z, void *p, const FcgScalars *s, hipStream_t st);

}  // namespace hisq
