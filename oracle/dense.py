"""Dense matrix of the staggered HISQ Dslash on a tiny lattice.

TEST INFRASTRUCTURE ONLY.  The matrix is assembled block by block from the
stencil of the paper's Sec. 5.1 (with Kogut-Susskind phases and the spinor
boundary conditions of Sec. 3): for every site and every hop (+-1, +-3 along
each direction) the 3x3 colour block it contributes is written into the
(3V x 3V) matrix.  It is meant for lattices up to 4^4 (768 x 768).
"""
from __future__ import annotations

import numpy as np


def dense_dslash(dims, t_bc: int, X, W) -> np.ndarray:
    """Return the (3V, 3V) complex matrix D with (D psi) = D @ psi.ravel()."""
    nx, ny, nz, nt = (int(d) for d in dims)
    shape = (nt, nz, ny, nx)  # lexicographic order, x fastest
    V = nx * ny * nz * nt
    ext = (nx, ny, nz, nt)
    Xl = np.asarray(X).reshape(4, V, 3, 3)
    Wl = np.asarray(W).reshape(4, V, 3, 3)
    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    for s in range(V):
        t, z, y, x = np.unravel_index(s, shape)
        xs = (int(x), int(y), int(z), int(t))
        for mu in range(4):
            eta = (-1) ** (sum(xs[:mu]) % 2)
            for k in (+1, -1, +3, -3):
                raw = xs[mu] + k
                wraps = raw < 0 or raw >= ext[mu]
                bc = t_bc if (mu == 3 and wraps) else 1
                nb = list(xs)
                nb[mu] = raw % ext[mu]
                n = int(np.ravel_multi_index((nb[3], nb[2], nb[1], nb[0]), shape))
                if k == +1:
                    block = Xl[mu, s]
                elif k == +3:
                    block = Wl[mu, s]
                elif k == -1:
                    block = -Xl[mu, n].conj().T
                else:
                    block = -Wl[mu, n].conj().T
                D[3 * s:3 * s + 3, 3 * n:3 * n + 3] += eta * bc * block
    return D


def parity_blocks(dims, D: np.ndarray):
    """Split D into (D_ee, D_eo, D_oe, D_oo) blocks in even/odd site order."""
    nx, ny, nz, nt = (int(d) for d in dims)
    V = nx * ny * nz * nt
    t, z, y, x = np.unravel_index(np.arange(V), (nt, nz, ny, nx))
    par = (x + y + z + t) % 2
    ev = np.nonzero(par == 0)[0]
    od = np.nonzero(par == 1)[0]
    ie = (3 * ev[:, None] + np.arange(3)).ravel()
    io = (3 * od[:, None] + np.arange(3)).ravel()
    return D[np.ix_(ie, ie)], D[np.ix_(ie, io)], D[np.ix_(io, ie)], D[np.ix_(io, io)]


def dense_normal_even(dims, t_bc: int, X, W, mass: float) -> np.ndarray:
    """M_e = m^2 - D_eo D_oe as a dense matrix on the even sites."""
    _, Deo, Doe, _ = parity_blocks(dims, dense_dslash(dims, t_bc, X, W))
    n = Deo.shape[0]
    return mass * mass * np.eye(n) - Deo @ Doe
