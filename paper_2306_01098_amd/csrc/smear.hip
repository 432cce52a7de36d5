// HISQ link smearing: thin links U -> fat links X and Naik links W, both in
// the canonical complex128 layout (4, Nt, Nz, Ny, Nx, 3, 3), ready for
// hisq_pack_links.  Two levels of smearing with a projection to U(3) between
// them (the HISQ treatment of Sec. 3.1).  FP64 throughout.
//
// One smearing level F = c1 L + c3 S3 + c5 S5 + c7 S7 + cL Lepage is built
// from nested staples in three passes, all links periodic:
//   T_{+nu}[A]_mu(x) = L_nu(x) A_mu(x+nu) L_nu(x+mu)^+
//   T_{-nu}[A]_mu(x) = L_nu(x-nu)^+ A_mu(x-nu) L_nu(x-nu+mu)
//   pass 1: S1[mu][nu,s] = T_{s nu}[L]_mu                 (24 fields)
//   pass 2: Q[mu][nu] = sum_{rho not mu,nu} sum_r T_{r rho}[c5 L_mu + c7 P_sigma]
//           with P_sigma = S1[mu][sigma,+] + S1[mu][sigma,-], sigma the
//           fourth direction                                  (12 fields)
//   pass 3: F_mu = c1 L_mu + sum_{nu,s} T_{s nu}[c3 L_mu + Q[mu][nu] + cL S1[mu][nu,s]]
// which expands to the 6 three-link, 24 five-link, 48 seven-link and 6 Lepage
// paths.  These are one-off per gauge field, so the passes favour clarity
// (one thread per output matrix, matrices stored whole) over bandwidth.
#include <cmath>
#include <cstdint>

#include "api_util.hpp"
#include "internal.hpp"

namespace hisq {

namespace {

constexpr int SB = 256;

struct M3 {
    double2 e[9];  // row-major, (re, im)
};

__device__ __forceinline__ M3 ldm(const double *base, size_t idx) {
    const double2 *p = reinterpret_cast<const double2 *>(base) + idx * 9;
    M3 m;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        m.e[k] = p[k];
    return m;
}

__device__ __forceinline__ void stm(double *base, size_t idx, const M3 &m) {
    double2 *p = reinterpret_cast<double2 *>(base) + idx * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        p[k] = m.e[k];
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmul_conj_b(double2 a, double2 b) {  // a conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cmul_conj_a(double2 a, double2 b) {  // conj(a) b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// A B
__device__ __forceinline__ M3 mul(const M3 &a, const M3 &b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double2 t = cmul(a.e[3 * i + k], b.e[3 * k + j]);
                s.x += t.x;
                s.y += t.y;
            }
            c.e[3 * i + j] = s;
        }
    return c;
}

// A B^+
__device__ __forceinline__ M3 mul_adj(const M3 &a, const M3 &b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double2 t = cmul_conj_b(a.e[3 * i + k], b.e[3 * j + k]);
                s.x += t.x;
                s.y += t.y;
            }
            c.e[3 * i + j] = s;
        }
    return c;
}

// A^+ B
__device__ __forceinline__ M3 adj_mul(const M3 &a, const M3 &b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double2 t = cmul_conj_a(a.e[3 * k + i], b.e[3 * k + j]);
                s.x += t.x;
                s.y += t.y;
            }
            c.e[3 * i + j] = s;
        }
    return c;
}

__device__ __forceinline__ void axpy(double a, const M3 &x, M3 &y) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        y.e[k].x = fma(a, x.e[k].x, y.e[k].x);
        y.e[k].y = fma(a, x.e[k].y, y.e[k].y);
    }
}

__device__ __forceinline__ M3 zero3() {
    M3 m;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        m.e[k] = make_double2(0.0, 0.0);
    return m;
}

struct Lat {
    int n[4];  // Nx, Ny, Nz, Nt
    int64_t V;
};

__device__ __forceinline__ void coords(const Lat &g, int64_t lex, int c[4]) {
    c[0] = (int)(lex % g.n[0]);
    lex /= g.n[0];
    c[1] = (int)(lex % g.n[1]);
    lex /= g.n[1];
    c[2] = (int)(lex % g.n[2]);
    c[3] = (int)(lex / g.n[2]);
}

__device__ __forceinline__ int64_t lex_of(const Lat &g, const int c[4]) {
    return c[0] + (int64_t)g.n[0] * (c[1] + (int64_t)g.n[1] * (c[2] + (int64_t)g.n[2] * c[3]));
}

// lex of site c + k * unit(d) (periodic)
__device__ __forceinline__ int64_t shift(const Lat &g, const int c[4], int d, int k) {
    int s[4] = {c[0], c[1], c[2], c[3]};
    s[d] = ((s[d] + k) % g.n[d] + g.n[d]) % g.n[d];
    return lex_of(g, s);
}

// The k-th direction (k = 0, 1, 2) other than mu.
__device__ __forceinline__ int other(int mu, int k) { return k < mu ? k : k + 1; }

// Index (0..2) of direction nu among the directions other than mu.
__device__ __forceinline__ int other_index(int mu, int nu) { return nu < mu ? nu : nu - 1; }

// Staple T_{s nu}[A]_mu(x) of the field whose value at site y is A(y).
template <typename F>
__device__ __forceinline__ M3 staple(const Lat &g, const double *L, const int c[4], int mu, int nu, int s, F A) {
    if (s > 0) {
        const int64_t xn = shift(g, c, nu, 1);
        const int64_t xm = shift(g, c, mu, 1);
        const M3 a = ldm(L, (size_t)nu * g.V + lex_of(g, c));
        const M3 b = A(xn);
        const M3 d = ldm(L, (size_t)nu * g.V + xm);
        return mul_adj(mul(a, b), d);
    }
    int cm[4] = {c[0], c[1], c[2], c[3]};
    cm[nu] = (cm[nu] - 1 + g.n[nu]) % g.n[nu];
    const int64_t xmn = lex_of(g, cm);
    const int64_t xmnm = shift(g, cm, mu, 1);
    const M3 a = ldm(L, (size_t)nu * g.V + xmn);
    const M3 b = A(xmn);
    const M3 d = ldm(L, (size_t)nu * g.V + xmnm);
    return mul(adj_mul(a, b), d);
}

// pass 1: S1[(mu * 6 + 2 k + (s < 0)) V + x] = T_{s nu_k}[L]_mu(x)
__global__ void __launch_bounds__(SB) staple1_kernel(Lat g, const double *L, double *S1) {
    const int64_t gid = (int64_t)blockIdx.x * SB + threadIdx.x;
    if (gid >= 24 * g.V)
        return;
    const int f = (int)(gid / g.V);
    const int64_t x = gid - (int64_t)f * g.V;
    const int mu = f / 6, j = f % 6;
    const int nu = other(mu, j >> 1), s = (j & 1) ? -1 : 1;
    int c[4];
    coords(g, x, c);
    const M3 r = staple(g, L, c, mu, nu, s, [&](int64_t y) { return ldm(L, (size_t)mu * g.V + y); });
    stm(S1, (size_t)f * g.V + x, r);
}

// pass 2: Q[(mu * 3 + k) V + x] for nu = nu_k
__global__ void __launch_bounds__(SB) staple2_kernel(Lat g, const double *L, const double *S1, double *Q,
                                                      double c5, double c7) {
    const int64_t gid = (int64_t)blockIdx.x * SB + threadIdx.x;
    if (gid >= 12 * g.V)
        return;
    const int f = (int)(gid / g.V);
    const int64_t x = gid - (int64_t)f * g.V;
    const int mu = f / 3, nu = other(mu, f % 3);
    int c[4];
    coords(g, x, c);
    M3 acc = zero3();
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        const int rho = other(mu, k);
        if (rho == nu)
            continue;
        const int sig = 6 - mu - nu - rho;
        const int js = other_index(mu, sig);
        auto Z = [&](int64_t y) {
            M3 z = zero3();
            axpy(c5, ldm(L, (size_t)mu * g.V + y), z);
            axpy(c7, ldm(S1, (size_t)(mu * 6 + 2 * js) * g.V + y), z);
            axpy(c7, ldm(S1, (size_t)(mu * 6 + 2 * js + 1) * g.V + y), z);
            return z;
        };
        axpy(1.0, staple(g, L, c, mu, rho, 1, Z), acc);
        axpy(1.0, staple(g, L, c, mu, rho, -1, Z), acc);
    }
    stm(Q, (size_t)f * g.V + x, acc);
}

// pass 3: F_mu(x)
__global__ void __launch_bounds__(SB) staple3_kernel(Lat g, const double *L, const double *S1, const double *Q,
                                                      double *F, double c1, double c3, double cl) {
    const int64_t gid = (int64_t)blockIdx.x * SB + threadIdx.x;
    if (gid >= 4 * g.V)
        return;
    const int mu = (int)(gid / g.V);
    const int64_t x = gid - (int64_t)mu * g.V;
    int c[4];
    coords(g, x, c);
    M3 acc = zero3();
    axpy(c1, ldm(L, (size_t)mu * g.V + x), acc);
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        const int nu = other(mu, k);
#pragma unroll 1
        for (int sj = 0; sj < 2; ++sj) {
            const int s = sj ? -1 : 1;
            auto A = [&](int64_t y) {
                M3 z = zero3();
                axpy(c3, ldm(L, (size_t)mu * g.V + y), z);
                axpy(1.0, ldm(Q, (size_t)(mu * 3 + k) * g.V + y), z);
                if (cl != 0.0)
                    axpy(cl, ldm(S1, (size_t)(mu * 6 + 2 * k + sj) * g.V + y), z);
                return z;
            };
            axpy(1.0, staple(g, L, c, mu, nu, s, A), acc);
        }
    }
    stm(F, (size_t)mu * g.V + x, acc);
}

// Y = V (V^+ V)^(-1/2).  The eigenvalues g_i of the Hermitian Q = V^+ V come
// from the trigonometric solution of its characteristic cubic; with
// s_i = sqrt(g_i), u = s0 + s1 + s2, v = s0 s1 + s0 s2 + s1 s2, w = s0 s1 s2,
// the quadratic f0 + f1 Q + f2 Q^2 that equals g^(-1/2) on the spectrum is
// f0 = (u v^2 - w (u^2 + v)) / D, f1 = (2 u v - u^3 - w) / D, f2 = u / D,
// D = w (u v - w): symmetric in the eigenvalues, so degenerate spectra are
// harmless (Hasenfratz, Hoffmann and Schaefer, JHEP 0705:029).
__global__ void __launch_bounds__(SB) project_kernel(int64_t n, const double *Vin, double *Y) {
    const int64_t i = (int64_t)blockIdx.x * SB + threadIdx.x;
    if (i >= n)
        return;
    const M3 v = ldm(Vin, (size_t)i);
    const M3 q = adj_mul(v, v);
    const double q00 = q.e[0].x, q11 = q.e[4].x, q22 = q.e[8].x;
    const double2 q01 = q.e[1], q02 = q.e[2], q12 = q.e[5];
    const double p1 = q01.x * q01.x + q01.y * q01.y + q02.x * q02.x + q02.y * q02.y + q12.x * q12.x +
                      q12.y * q12.y;
    const double tr = (q00 + q11 + q22) / 3.0;
    double g0, g1, g2;
    const double d0 = q00 - tr, d1 = q11 - tr, d2 = q22 - tr;
    const double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1;
    if (p2 <= 1e-30 * tr * tr) {
        g0 = g1 = g2 = tr;
    } else {
        const double p = sqrt(p2 / 6.0);
        // det(B) / 2 with B = (Q - tr 1) / p (Hermitian, so the determinant is real)
        const double b00 = d0 / p, b11 = d1 / p, b22 = d2 / p;
        const double2 b01 = make_double2(q01.x / p, q01.y / p), b02 = make_double2(q02.x / p, q02.y / p),
                      b12 = make_double2(q12.x / p, q12.y / p);
        const double n01 = b01.x * b01.x + b01.y * b01.y, n02 = b02.x * b02.x + b02.y * b02.y,
                     n12 = b12.x * b12.x + b12.y * b12.y;
        // 2 Re(b01 b12 conj(b02))
        const double2 t = cmul(b01, b12);
        const double tri = 2.0 * (t.x * b02.x + t.y * b02.y);
        double r = 0.5 * (b00 * b11 * b22 + tri - b00 * n12 - b11 * n02 - b22 * n01);
        r = fmin(1.0, fmax(-1.0, r));
        const double phi = acos(r) / 3.0;
        g0 = tr + 2.0 * p * cos(phi);
        g2 = tr + 2.0 * p * cos(phi + 2.0943951023931954923);  // + 2 pi / 3
        g1 = 3.0 * tr - g0 - g2;
    }
    const double s0 = sqrt(fmax(g0, 0.0)), s1 = sqrt(fmax(g1, 0.0)), s2 = sqrt(fmax(g2, 0.0));
    const double u = s0 + s1 + s2, vv = s0 * s1 + s0 * s2 + s1 * s2, w = s0 * s1 * s2;
    const double den = w * (u * vv - w);
    const double f0 = (u * vv * vv - w * (u * u + vv)) / den;
    const double f1 = (2.0 * u * vv - u * u * u - w) / den;
    const double f2 = u / den;
    const M3 q2 = mul(q, q);
    M3 h = zero3();
    h.e[0].x = h.e[4].x = h.e[8].x = f0;
    axpy(f1, q, h);
    axpy(f2, q2, h);
    stm(Y, (size_t)i, mul(v, h));
}

// W_mu(x) = c Y_mu(x) Y_mu(x + mu) Y_mu(x + 2 mu)
__global__ void __launch_bounds__(SB) naik_kernel(Lat g, const double *Y, double *W, double cn) {
    const int64_t gid = (int64_t)blockIdx.x * SB + threadIdx.x;
    if (gid >= 4 * g.V)
        return;
    const int mu = (int)(gid / g.V);
    const int64_t x = gid - (int64_t)mu * g.V;
    int c[4];
    coords(g, x, c);
    const M3 a = ldm(Y, (size_t)mu * g.V + x);
    const M3 b = ldm(Y, (size_t)mu * g.V + shift(g, c, mu, 1));
    const M3 d = ldm(Y, (size_t)mu * g.V + shift(g, c, mu, 2));
    M3 r = mul(mul(a, b), d);
    M3 out = zero3();
    axpy(cn, r, out);
    stm(W, (size_t)mu * g.V + x, out);
}

unsigned blocks(int64_t n) { return (unsigned)((n + SB - 1) / SB); }

struct SmearLayout {
    size_t v, y, s1, q, total;
};

SmearLayout smear_layout(int64_t V) {
    const size_t mat = 144;
    SmearLayout L;
    L.v = 0;
    L.y = L.v + 4 * V * mat;
    L.s1 = L.y + 4 * V * mat;
    L.q = L.s1 + 24 * V * mat;
    L.total = L.q + 12 * V * mat;
    return L;
}

hipError_t smear_level(const Lat &g, const double *L, double *S1, double *Q, double *F, double c1, double c3,
                       double c5, double c7, double cl, hipStream_t st) {
    staple1_kernel<<<blocks(24 * g.V), SB, 0, st>>>(g, L, S1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    staple2_kernel<<<blocks(12 * g.V), SB, 0, st>>>(g, L, S1, Q, c5, c7);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    staple3_kernel<<<blocks(4 * g.V), SB, 0, st>>>(g, L, S1, Q, F, c1, c3, cl);
    return hipGetLastError();
}

}  // namespace

}  // namespace hisq

using namespace hisq;

extern "C" {

size_t hisq_smear_workspace_bytes(const hisq_lattice *lat) {
    if (check_lattice(lat) != HISQ_OK)
        return 0;
    const int64_t V = (int64_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
    return smear_layout(V).total;
}

hisq_status hisq_smear_links(hisq_context *ctx, const hisq_lattice *lat, const void *thin_c128, double naik_eps,
                             void *fat_c128, void *naik_c128, void *ws, size_t ws_bytes, void *stream) {
    TRY(check_lattice(lat));
    TRY(check_ptr(thin_c128, "thin_c128"));
    TRY(check_ptr(fat_c128, "fat_c128"));
    TRY(check_ptr(naik_c128, "naik_c128"));
    TRY(check_ptr(ws, "ws"));
    if (fat_c128 == naik_c128 || fat_c128 == thin_c128 || naik_c128 == thin_c128)
        return fail(HISQ_ERR_INVALID_ARG, "thin, fat and naik buffers must be distinct");
    if (!std::isfinite(naik_eps))
        return fail(HISQ_ERR_INVALID_ARG, "naik_eps must be finite");
    Lat g;
    for (int d = 0; d < 4; ++d)
        g.n[d] = lat->dims[d];
    g.V = (int64_t)g.n[0] * g.n[1] * g.n[2] * g.n[3];
    const SmearLayout L = smear_layout(g.V);
    if (ws_bytes < L.total)
        return fail(HISQ_ERR_WORKSPACE, "workspace holds %zu bytes, needs %zu", ws_bytes, L.total);
    TRY(set_device(ctx));
    const hipStream_t st = static_cast<hipStream_t>(stream);
    char *W = static_cast<char *>(ws);
    double *V1 = reinterpret_cast<double *>(W + L.v);
    double *Y = reinterpret_cast<double *>(W + L.y);
    double *S1 = reinterpret_cast<double *>(W + L.s1);
    double *Q = reinterpret_cast<double *>(W + L.q);
    const double *U = static_cast<const double *>(thin_c128);
    // level 1 (fat7), projection, level 2 (fat7 + Lepage), Naik
    hipError_t e = smear_level(g, U, S1, Q, V1, 1.0 / 8, 1.0 / 16, 1.0 / 64, 1.0 / 384, 0.0, st);
    if (e == hipSuccess) {
        project_kernel<<<blocks(4 * g.V), SB, 0, st>>>(4 * g.V, V1, Y);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = smear_level(g, Y, S1, Q, static_cast<double *>(fat_c128), 1.0, 1.0 / 16, 1.0 / 64, 1.0 / 384,
                        -1.0 / 8, st);
    if (e == hipSuccess) {
        naik_kernel<<<blocks(4 * g.V), SB, 0, st>>>(g, Y, static_cast<double *>(naik_c128),
                                                      -1.0 / 24 + naik_eps / 8);
        e = hipGetLastError();
    }
    return e == hipSuccess ? HISQ_OK : device_fail(e, "smear_links");
}

}  // extern "C"
