"""Seeded synthetic inputs for the HISQ Dslash / CG path.

This module only draws random gauge fields, sources and masses and lays them
out in the canonical host-side formats.  It holds none of the method's
arithmetic (no stencil, no solver), so both the FP64 oracle and the GPU path
may consume what it produces.

Canonical formats (complex128, interleaved re/im):

* links ``(4, Nt, Nz, Ny, Nx, 3, 3)``: entry ``[mu, t, z, y, x, row, col]`` is
  the 3x3 link matrix leaving site (x, y, z, t) in direction mu, x fastest
  (the lexicographic order of the paper's indexing section).
* half-lattice fields ``(nrhs, V/2, 3)``: the colour vectors on the sites of
  one parity, in increasing lexicographic order (equivalently the index
  floor(lex/2) of the paper's even/odd formula).

Generators
----------
* Haar SU(3): QR of a complex Ginibre matrix with the phases of diag(R) moved
  into Q (Mezzadri, "How to generate random matrices from the classical compact
  groups", 2007), times det(Q)^(-1/3).
* Smooth links: U = exp(i eps H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0,1)
  and lambda_a the Gell-Mann matrices, evaluated through the eigendecomposition
  of H.
* Long (Naik-like) links: W_mu(x) = V_mu(x) V_mu(x+mu) V_mu(x+2mu) for a third
  smooth field V (periodic gauge boundary).
* Sources: real and imaginary parts ~ N(0, 1/2), so E|z|^2 = 1.

Seeds: ``seed = 1000*k + field_id`` with fat 1, long 2, source 3+i,
masses 4, gauge transform 5 (k is the workload number).
"""
from __future__ import annotations

import numpy as np
import torch

FIELD_FAT, FIELD_LONG, FIELD_SOURCE, FIELD_MASS, FIELD_GAUGE = 1, 2, 3, 4, 5


def rng_for(k: int, field_id: int) -> np.random.Generator:
    """PCG64 generator for workload ``k`` and field ``field_id``."""
    return np.random.Generator(np.random.PCG64(1000 * k + field_id))


def volume(dims) -> int:
    nx, ny, nz, nt = dims
    return int(nx) * int(ny) * int(nz) * int(nt)


def _ginibre(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, 3, 3, 2))
    return (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)


def haar_su3(rng: np.random.Generator, n: int) -> np.ndarray:
    """``n`` Haar-distributed SU(3) matrices, shape (n, 3, 3) complex128."""
    z = torch.from_numpy(_ginibre(rng, n))
    q, r = torch.linalg.qr(z)
    d = torch.diagonal(r, dim1=-2, dim2=-1)
    ph = d / d.abs()
    q = q * ph[:, None, :]
    det = torch.linalg.det(q)
    q = q * torch.exp(-1j * torch.angle(det) / 3.0)[:, None, None]
    return q.numpy()


_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1], _GELL_MANN[1][1, 0] = -1j, 1j
_GELL_MANN[2][0, 0], _GELL_MANN[2][1, 1] = 1, -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2], _GELL_MANN[4][2, 0] = -1j, 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2], _GELL_MANN[6][2, 1] = -1j, 1j
_GELL_MANN[7][0, 0] = _GELL_MANN[7][1, 1] = 1 / np.sqrt(3)
_GELL_MANN[7][2, 2] = -2 / np.sqrt(3)


def smooth_su3(rng: np.random.Generator, n: int, eps: float) -> np.ndarray:
    """``n`` matrices exp(i eps H), H Gaussian Hermitian traceless (n, 3, 3)."""
    h = rng.standard_normal((n, 8))
    H = torch.from_numpy(np.einsum("na,aij->nij", h, _GELL_MANN / 2.0))
    w, v = torch.linalg.eigh(H)
    u = (v * torch.exp(1j * eps * w)[:, None, :]) @ v.conj().transpose(1, 2)
    return u.numpy()


def _as_links(mats: np.ndarray, dims) -> np.ndarray:
    nx, ny, nz, nt = dims
    return np.ascontiguousarray(mats.reshape(4, nt, nz, ny, nx, 3, 3))


# axis of the (Nt, Nz, Ny, Nx) site block that direction mu moves along
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def haar_links(dims, rng: np.random.Generator) -> np.ndarray:
    return _as_links(haar_su3(rng, 4 * volume(dims)), dims)


def smooth_links(dims, rng: np.random.Generator, eps: float) -> np.ndarray:
    return _as_links(smooth_su3(rng, 4 * volume(dims), eps), dims)


def long_links_from(v: np.ndarray) -> np.ndarray:
    """W_mu(x) = V_mu(x) V_mu(x+mu) V_mu(x+2mu), periodic gauge boundary."""
    w = np.empty_like(v)
    for mu in range(4):
        ax = _AXIS[mu]
        v0 = torch.from_numpy(v[mu])
        v1 = torch.from_numpy(np.roll(v[mu], -1, axis=ax))
        v2 = torch.from_numpy(np.roll(v[mu], -2, axis=ax))
        w[mu] = (v0 @ v1 @ v2).numpy()
    return w


def gaussian_half_field(rng: np.random.Generator, dims, nrhs: int = 1) -> np.ndarray:
    """(nrhs, V/2, 3) complex source with Re, Im ~ N(0, 1/2)."""
    n = volume(dims) // 2
    g = rng.standard_normal((nrhs, n, 3, 2)) * np.sqrt(0.5)
    return g[..., 0] + 1j * g[..., 1]


def gaussian_full_field(rng: np.random.Generator, dims) -> np.ndarray:
    """(Nt, Nz, Ny, Nx, 3) complex field with Re, Im ~ N(0, 1/2)."""
    nx, ny, nz, nt = dims
    g = rng.standard_normal((nt, nz, ny, nx, 3, 2)) * np.sqrt(0.5)
    return g[..., 0] + 1j * g[..., 1]


def gauge_transform(dims, rng: np.random.Generator) -> np.ndarray:
    """Haar SU(3) matrix per site, shape (Nt, Nz, Ny, Nx, 3, 3)."""
    nx, ny, nz, nt = dims
    return haar_su3(rng, volume(dims)).reshape(nt, nz, ny, nx, 3, 3)


# ---------------------------------------------------------------------------
# The five workloads.  Each returns a dict of host numpy arrays + parameters.
# ---------------------------------------------------------------------------

def workload_haar(dims, k: int, t_bc: int, nsrc: int = 1):
    """Haar-random fat and long links, Gaussian even-site sources."""
    return dict(
        dims=tuple(dims), t_bc=t_bc,
        fat=haar_links(dims, rng_for(k, FIELD_FAT)),
        naik=haar_links(dims, rng_for(k, FIELD_LONG)),
        src=gaussian_half_field(rng_for(k, FIELD_SOURCE), dims, nsrc),
    )


def workload_smooth(dims, k: int, t_bc: int, eps: float = 0.3, nsrc: int = 1,
                    src_offset: int = 0):
    """Smooth fat links exp(i eps H), long links as 3-link path products."""
    fat = smooth_links(dims, rng_for(k, FIELD_FAT), eps)
    v = smooth_links(dims, rng_for(k, FIELD_LONG), eps)
    return dict(dims=tuple(dims), t_bc=t_bc, fat=fat, naik=long_links_from(v),
                src=gaussian_half_field(rng_for(k, FIELD_SOURCE + src_offset), dims, nsrc))


def workload_1():
    """8^4, periodic time boundary, Haar links, one source, m = 0.1."""
    w = workload_haar((8, 8, 8, 8), 1, +1)
    w["mass"] = 0.1
    return w


def workload_2(dims=(32, 32, 32, 8)):
    """32^3x8 smooth links eps=0.3, antiperiodic time, m = 0.01."""
    w = workload_smooth(dims, 2, -1, 0.3)
    w["mass"] = 0.01
    return w


def workload_3(dims=(48, 48, 48, 12), nsrc: int = 16):
    """48^3x12 smooth links, 16 sources, m = 0.005, 14 log-spaced shifts."""
    w = workload_smooth(dims, 3, -1, 0.3, nsrc=nsrc)
    w["mass"] = 0.005
    w["shifts"] = 10.0 ** (-5.0 + 5.0 * np.arange(14) / 13.0)
    return w


BATCH_MIX = (((8, 8, 8, 8), 24), ((12, 12, 12, 4), 20), ((16, 16, 16, 8), 12),
             ((24, 24, 24, 6), 8))


def workload_4(mix=BATCH_MIX):
    """Uneven batch: independent Haar lattices, masses ~ U[0.01, 0.1]."""
    probs = []
    mrng = rng_for(4, FIELD_MASS)
    j = 0
    for dims, count in mix:
        for _ in range(count):
            probs.append(dict(workload_haar(dims, 4000 + j, -1), mass=float(mrng.uniform(0.01, 0.1))))
            j += 1
    return probs


def workload_5(dims=(32, 32, 32, 32), ntrain: int = 256, ntest: int = 16):
    """32^4 smooth links eps=0.3, m = 0.005, training and held-out sources."""
    w = workload_smooth(dims, 5, -1, 0.3, nsrc=0)
    w["mass"] = 0.005
    w["train_src"] = gaussian_half_field(rng_for(5, FIELD_SOURCE), dims, ntrain)
    w["test_src"] = gaussian_half_field(rng_for(5, FIELD_SOURCE + 1), dims, ntest)
    return w


PTC_CHANNELS = (1, 8, 8, 1)
PTC_PATHS = 9


def ptc_initial_weights(seed: int, scale: float = 0.05):
    """Seeded starting weights of the 1 -> 8 -> 8 -> 1 PTC network, one
    (c_out, c_in, 9) complex array per layer: the identity path starts at
    1/sqrt(c_in c_out), every weight gets complex Gaussian noise of width
    scale/sqrt(9 c_in).  A random draw only (the network itself is elsewhere)."""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in zip(PTC_CHANNELS[:-1], PTC_CHANNELS[1:]):
        g = rng.standard_normal((cout, cin, PTC_PATHS, 2)) * scale / np.sqrt(cin * PTC_PATHS)
        w = g[..., 0] + 1j * g[..., 1]
        w[:, :, 0] += 1.0 / np.sqrt(cin * cout)
        out.append(w)
    return out
