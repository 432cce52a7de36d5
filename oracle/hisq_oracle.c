/*
 * FP64 CPU oracle for the HISQ staggered Dslash.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU library: it works on whole-lattice fields in lexicographic site
 * order with C99 complex arithmetic, one output site at a time, exactly as the
 * operator is written down.
 *
 * The operator (paper, Sec. 5.1 "HISQ Dslash performance model", the stencil
 * equation there; lattice and boundary conditions from Sec. 3 "Physics
 * modules"; staggered phases of Kogut and Susskind, which the paper omits for
 * convenience):
 *
 *   (D psi)(x) = sum_{mu=0..3} eta_mu(x) [ X_mu(x) psi(x+mu)  - X_mu(x-mu)^+  psi(x-mu)
 *                                        + W_mu(x) psi(x+3mu) - W_mu(x-3mu)^+ psi(x-3mu) ]
 *
 *   eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z)
 *
 * Neighbour coordinates are taken modulo the extent; a hop that wraps around
 * the lattice in direction mu picks up the spinor boundary sign bc_mu
 * (+1 in space, t_bc in time).  Readings where the printed formula is garbled:
 * the direction sum runs over the four directions 0..3, the forward three-hop
 * link is W_mu(x) (the link from x to x+3mu), and no overall constant.
 *
 * Layouts (all complex128):
 *   links  [mu][site][row][col], site = x + Nx*(y + Ny*(z + Nz*t))
 *   fields [site][colour]
 */
#include <complex.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static long site_of(const int c[4], const int n[4])
{
    return (long)c[0] + (long)n[0] * ((long)c[1] + (long)n[1] * ((long)c[2] + (long)n[2] * (long)c[3]));
}

static void coords_of(long s, const int n[4], int c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(s % n[mu]);
        s /= n[mu];
    }
}

/* Move the site with coordinates c by k steps along mu.  Writes the neighbour
 * coordinates into d and returns the boundary sign of the hop. */
static double hop(const int c[4], const int n[4], int mu, int k, int t_bc, int d[4])
{
    for (int nu = 0; nu < 4; ++nu)
        d[nu] = c[nu];
    int v = c[mu] + k;
    double sign = 1.0;
    if (v >= n[mu] || v < 0) {
        v = ((v % n[mu]) + n[mu]) % n[mu];
        if (mu == 3)
            sign = (double)t_bc;
    }
    d[mu] = v;
    return sign;
}

/* y += s * U psi */
static void mul_add(cplx y[3], double s, const cplx *U, const cplx *psi)
{
    for (int a = 0; a < 3; ++a) {
        cplx acc = 0;
        for (int b = 0; b < 3; ++b)
            acc += U[3 * a + b] * psi[b];
        y[a] += s * acc;
    }
}

/* y += s * U^+ psi */
static void mul_adj_add(cplx y[3], double s, const cplx *U, const cplx *psi)
{
    for (int a = 0; a < 3; ++a) {
        cplx acc = 0;
        for (int b = 0; b < 3; ++b)
            acc += conj(U[3 * b + a]) * psi[b];
        y[a] += s * acc;
    }
}

static double eta(const int c[4], int mu)
{
    int s = 0;
    for (int nu = 0; nu < mu; ++nu)
        s += c[nu];
    return (s & 1) ? -1.0 : 1.0;
}

/* (D psi)(s) for one site s, written into acc[3]. */
static void site_dslash(const int dims[4], long V, int t_bc, const cplx *X, const cplx *W,
                        const cplx *psi, long s, cplx acc[3])
{
    int c[4], d[4];
    coords_of(s, dims, c);
    acc[0] = acc[1] = acc[2] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        const double e = eta(c, mu);
        double sg;
        long nb;
        /* one-hop forward: X_mu(x) psi(x+mu) */
        sg = hop(c, dims, mu, +1, t_bc, d);
        nb = site_of(d, dims);
        mul_add(acc, e * sg, &X[((long)mu * V + s) * 9], &psi[nb * 3]);
        /* one-hop backward: -X_mu(x-mu)^+ psi(x-mu) */
        sg = hop(c, dims, mu, -1, t_bc, d);
        nb = site_of(d, dims);
        mul_adj_add(acc, -e * sg, &X[((long)mu * V + nb) * 9], &psi[nb * 3]);
        /* three-hop forward: W_mu(x) psi(x+3mu) */
        sg = hop(c, dims, mu, +3, t_bc, d);
        nb = site_of(d, dims);
        mul_add(acc, e * sg, &W[((long)mu * V + s) * 9], &psi[nb * 3]);
        /* three-hop backward: -W_mu(x-3mu)^+ psi(x-3mu) */
        sg = hop(c, dims, mu, -3, t_bc, d);
        nb = site_of(d, dims);
        mul_adj_add(acc, -e * sg, &W[((long)mu * V + nb) * 9], &psi[nb * 3]);
    }
}

static int dims_ok(const int dims[4])
{
    for (int mu = 0; mu < 4; ++mu)
        if (dims[mu] <= 0)
            return 0;
    return 1;
}

/*
 * out = D psi on the whole lattice.  If out_parity is 0 or 1, only sites of
 * that parity are computed and the other sites of out are set to zero.
 * Returns 0, or -1 if an extent is not positive.
 */
int oracle_dslash(const int dims[4], int t_bc, const cplx *X, const cplx *W,
                  const cplx *psi, cplx *out, int out_parity)
{
    if (!dims_ok(dims))
        return -1;
    const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        int c[4];
        coords_of(s, dims, c);
        const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
        cplx acc[3] = {0, 0, 0};
        if (out_parity < 0 || par == out_parity)
            site_dslash(dims, V, t_bc, X, W, psi, s, acc);
        for (int a = 0; a < 3; ++a)
            out[s * 3 + a] = acc[a];
    }
    return 0;
}

/*
 * Dslash at a list of output sites only (spot checks of large lattices).
 * sites[k] is a lexicographic site; out[k*3 + a] receives (D psi)(sites[k])_a.
 */
int oracle_dslash_sites(const int dims[4], int t_bc, const cplx *X, const cplx *W,
                        const cplx *psi, const long *sites, long nsites, cplx *out)
{
    if (!dims_ok(dims))
        return -1;
    const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nsites; ++k)
        site_dslash(dims, V, t_bc, X, W, psi, sites[k], &out[k * 3]);
    return 0;
}

/* Number of OpenMP threads the oracle will use (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of OpenMP threads of later calls (for timing the oracle on
 * one core); the results do not depend on it. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
