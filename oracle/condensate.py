"""FP64 oracle of the stochastic chiral-condensate estimator.

TEST INFRASTRUCTURE ONLY (tests, the smoke check, the benchmark's CPU
baseline).  Shares no code with the GPU library.

The paper lists the chiral condensate among its observables (Sec. 3.3) and
measures it with a small number of random vectors.  Definitions used here:

  pbp = (1/V) Tr (D + m)^-1                       (trace over sites and colour)

With D anti-Hermitian and parity-flipping, (D + m)^-1 = (m - D)(m^2 - D^2)^-1;
D (m^2 - D^2)^-1 has no diagonal parity blocks, so its trace vanishes, and the
odd-site block m^2 - D_oe D_eo has the spectrum of M_e = m^2 - D_eo D_oe.
Hence

  pbp = (2 m / V) Tr_e M_e^-1,

estimated with noise vectors eta_i on the even sites, E[eta eta^+] = 1:

  pbp ~ (1/N) sum_i s_i,   s_i = (2 m / V) Re <eta_i, M_e^-1 eta_i>,

with the standard error of the mean of the s_i as its statistical error.
"""
from __future__ import annotations

import numpy as np

from . import dense
from .hisq import Lattice, cg, volume


def exact_dense(dims, t_bc: int, X, W, mass: float) -> float:
    """(1/V) Tr (D + m)^-1 from the dense full-lattice matrix (4^4 at most)."""
    D = dense.dense_dslash(dims, t_bc, X, W)
    n = D.shape[0]
    return float(np.trace(np.linalg.inv(D + mass * np.eye(n))).real / volume(dims))


def exact_even(dims, t_bc: int, X, W, mass: float) -> float:
    """(2 m / V) Tr_e M_e^-1 from the dense even-site matrix (4^4 at most)."""
    M = dense.dense_normal_even(dims, t_bc, X, W, mass)
    return float(2.0 * mass * np.trace(np.linalg.inv(M)).real / volume(dims))


def free_field(dims, t_bc: int, a: float, b: float, mass: float) -> float:
    """Closed form for X = a 1, W = b 1: M_e has eigenvalue
    lambda(p) = m^2 + 4 sum_mu (a sin p_mu + b sin 3 p_mu)^2 on each class
    {p, p + (pi, pi, pi, pi)} of allowed momenta, three colours each, so
    Tr_e M_e^-1 = (3/2) sum_p 1/lambda(p) and pbp = (3 m / V) sum_p 1/lambda(p)."""
    axes = []
    for mu, n in enumerate(dims):
        k = np.arange(n)
        anti = mu == 3 and t_bc == -1
        axes.append((2 * k + 1) * np.pi / n if anti else 2 * np.pi * k / n)
    grids = np.meshgrid(*axes, indexing="ij")
    lam = mass * mass + 4 * sum((a * np.sin(p) + b * np.sin(3 * p)) ** 2 for p in grids)
    return float(3.0 * mass * np.sum(1.0 / lam) / volume(dims))


def samples(lat: Lattice, mass: float, noise, tol: float = 1e-12, max_iter: int = 100000) -> np.ndarray:
    """s_i = (2 m / V) Re <eta_i, M_e^-1 eta_i> with the oracle's CG."""
    V = volume(lat.dims)
    out = []
    for eta in noise:
        r = cg(lat, mass, eta, tol, max_iter)
        out.append(2.0 * mass * np.vdot(np.ravel(eta), np.ravel(r.x)).real / V)
    return np.array(out)


def estimate(s) -> tuple[float, float]:
    """Mean and standard error of the samples."""
    s = np.asarray(s, dtype=np.float64)
    err = float(s.std(ddof=1) / np.sqrt(len(s))) if len(s) > 1 else float("nan")
    return float(s.mean()), err
