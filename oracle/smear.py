"""FP64 oracle of HISQ link smearing (thin links U -> fat links X, Naik links W).

TEST INFRASTRUCTURE ONLY (tests, the smoke check, the benchmark's CPU
baseline).  Shares no code with the GPU library.

The paper's HISQ treatment (Sec. 3.1, its commented coefficient block) has two
levels of smearing:

  level 1 (fat7):  V = c1 U + c3 (3-link staples) + c5 (5-link) + c7 (7-link),
                   c1 = 1/8, c3 = 1/16, c5 = 1/64, c7 = 1/384;
  projection:      Y = V (V^+ V)^(-1/2)   (back to U(3));
  level 2:         X = c1 Y + c3 (3-link) + c5 (5-link) + c7 (7-link)
                       + c_Lepage (Lepage), all built from Y,
                   c1 = 1, c3 = 1/16, c5 = 1/64, c7 = 1/384, c_Lepage = -1/8;
  Naik:            W_mu(x) = c_Naik Y_mu(x) Y_mu(x+mu) Y_mu(x+2mu),
                   c_Naik = -1/24 + eps/8.

Staples (links periodic).  For a link field L and a "transported" field A,
the staple along +-nu of A_mu at x is

  T_{+nu}[A]_mu(x) = L_nu(x) A_mu(x+nu) L_nu(x+mu)^+
  T_{-nu}[A]_mu(x) = L_nu(x-nu)^+ A_mu(x-nu) L_nu(x-nu+mu)

3-link: sum over the 6 signed nu != mu of T_nu[L]; 5-link: T_nu[T_rho[L]] over
signed nu, rho with mu, nu, rho distinct (24 paths); 7-link: T_nu[T_rho[T_sigma[L]]]
over distinct mu, nu, rho, sigma (48 paths); Lepage: T_nu[T_nu[L]] with the
same signed direction twice (6 paths).  This module builds each sum directly
from its definition (nested staples over explicit index loops);
``path_sum_at`` multiplies the links of every path one by one as an
independent check.

Arrays are (4, Nt, Nz, Ny, Nx, 3, 3) complex128, x fastest.
"""
from __future__ import annotations

import itertools

import numpy as np

AXIS = {0: 3, 1: 2, 2: 1, 3: 0}      # array axis of (Nt, Nz, Ny, Nx) moved along by mu

LEVEL1 = dict(c1=1 / 8, c3=1 / 16, c5=1 / 64, c7=1 / 384, cl=0.0)
LEVEL2 = dict(c1=1.0, c3=1 / 16, c5=1 / 64, c7=1 / 384, cl=-1 / 8)


def _shift(a, mu, k):
    """a(x + k mu) for a site field a of shape (Nt, Nz, Ny, Nx, ...)."""
    return np.roll(a, -k, axis=AXIS[mu])


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def staple(L, A_mu, mu: int, nu: int, s: int):
    """T_{s nu}[A]_mu over the whole lattice (A_mu: one direction's field)."""
    if s > 0:
        return L[nu] @ _shift(A_mu, nu, 1) @ _dag(_shift(L[nu], mu, 1))
    Lm = _shift(L[nu], nu, -1)                      # L_nu(x - nu)
    return _dag(Lm) @ _shift(A_mu, nu, -1) @ _shift(Lm, mu, 1)


def smear_level(L, c1, c3, c5, c7, cl):
    """c1 L + c3 S3 + c5 S5 + c7 S7 + cl Lepage, all from the link field L."""
    out = np.empty_like(L)
    for mu in range(4):
        others = [d for d in range(4) if d != mu]
        acc = c1 * L[mu]
        for nu in others:
            for s in (1, -1):
                acc = acc + c3 * staple(L, L[mu], mu, nu, s)
                if cl != 0.0:
                    acc = acc + cl * staple(L, staple(L, L[mu], mu, nu, s), mu, nu, s)
                for rho in others:
                    if rho == nu:
                        continue
                    for r in (1, -1):
                        inner5 = staple(L, L[mu], mu, rho, r)
                        acc = acc + c5 * staple(L, inner5, mu, nu, s)
                        for sig in others:
                            if sig in (nu, rho):
                                continue
                            for q in (1, -1):
                                inner7 = staple(L, staple(L, L[mu], mu, sig, q), mu, rho, r)
                                acc = acc + c7 * staple(L, inner7, mu, nu, s)
        out[mu] = acc
    return out


def u3_project(V):
    """V (V^+ V)^(-1/2) per matrix, via the eigen-decomposition of V^+ V."""
    Q = _dag(V) @ V
    g, P = np.linalg.eigh(Q)
    inv_sqrt = (P * (1.0 / np.sqrt(g))[..., None, :]) @ _dag(P)
    return V @ inv_sqrt


def naik(Y, c_naik):
    out = np.empty_like(Y)
    for mu in range(4):
        out[mu] = c_naik * (Y[mu] @ _shift(Y[mu], mu, 1) @ _shift(Y[mu], mu, 2))
    return out


def hisq_smear(U, eps: float = 0.0):
    """(X, W) of the HISQ action from thin links U."""
    V = smear_level(U, **LEVEL1)
    Y = u3_project(V)
    X = smear_level(Y, **LEVEL2)
    W = naik(Y, -1.0 / 24.0 + eps / 8.0)
    return X, W


# ---------------------------------------------------------------------------
# Independent check: explicit path products at one site.
# ---------------------------------------------------------------------------
def _link(L, dims, x, mu):
    nx, ny, nz, nt = dims
    return L[mu, x[3] % nt, x[2] % nz, x[1] % ny, x[0] % nx]


def path_product(L, dims, x, steps):
    """Product of links along a path of signed unit steps (+-(d+1)) from x."""
    m = np.eye(3, dtype=np.complex128)
    pos = list(x)
    for st in steps:
        d = abs(st) - 1
        if st > 0:
            m = m @ _link(L, dims, pos, d)
            pos[d] += 1
        else:
            pos[d] -= 1
            m = m @ _dag(_link(L, dims, pos, d))
    return m


def staple_paths(mu: int, dirs):
    """Signed-step path of the nested staple T_{d1}[T_{d2}[...[L_mu]]] with
    dirs = (d1, d2, ...), each a signed direction +-(nu+1)."""
    return list(dirs) + [mu + 1] + [-d for d in reversed(dirs)]


def path_sum_at(L, dims, x, mu, c1, c3, c5, c7, cl):
    """The same smeared link at one site from explicit path products."""
    others = [d for d in range(4) if d != mu]
    signed = [s * (d + 1) for d in others for s in (1, -1)]
    acc = c1 * _link(L, dims, x, mu)
    for a in signed:
        acc = acc + c3 * path_product(L, dims, x, staple_paths(mu, (a,)))
        acc = acc + cl * path_product(L, dims, x, staple_paths(mu, (a, a)))
    for a, b in itertools.permutations(signed, 2):
        if abs(a) != abs(b):
            acc = acc + c5 * path_product(L, dims, x, staple_paths(mu, (a, b)))
    for a, b, c in itertools.permutations(signed, 3):
        if len({abs(a), abs(b), abs(c)}) == 3:
            acc = acc + c7 * path_product(L, dims, x, staple_paths(mu, (a, b, c)))
    return acc
