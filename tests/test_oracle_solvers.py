"""Pins of the oracle solvers: dense solves, closed forms, status codes."""
import itertools

import numpy as np
import pytest

import hisq_inputs as gen
from oracle import dense
from oracle import hisq as O


def test_cg_matches_dense_solve_4x4x4x4():
    dims = (4, 4, 4, 4)
    w = gen.workload_haar(dims, 21, -1)
    lat = O.lattice_from(w)
    m = 0.1
    b = w["src"][0]
    res = O.cg(lat, m, b, 1e-12, 2000)
    assert res.status == O.OK and res.true_residual <= 1e-12
    M = dense.dense_normal_even(dims, -1, w["fat"], w["naik"], m)
    xd = np.linalg.solve(M, b.ravel())
    kappa = np.linalg.cond(M)
    assert np.linalg.norm(res.x.ravel() - xd) <= 10 * kappa * 1e-12 * np.linalg.norm(xd)
    # the dense residual of the oracle's solution is tiny, independently of M_e
    assert np.linalg.norm(b.ravel() - M @ res.x.ravel()) <= 1e-12 * np.linalg.norm(b)


def test_cg_free_plane_wave_is_one_step():
    """P_e phi_p is an eigenvector of free M_e: x = b / lambda(p)."""
    dims = (4, 4, 4, 8)
    a, bcoef, m, t_bc = 1.0, -1.0 / 24, 0.2, -1
    nx, ny, nz, nt = dims
    X = np.zeros((4, nt, nz, ny, nx, 3, 3), complex)
    W = np.zeros_like(X)
    for c in range(3):
        X[..., c, c] = a
        W[..., c, c] = bcoef
    lat = O.Lattice(dims, t_bc, X, W)
    p = (2 * np.pi / 4, 2 * np.pi * 3 / 4, 0.0, 3 * np.pi / 8)
    t, z, y, x = np.meshgrid(*[np.arange(n) for n in (nt, nz, ny, nx)], indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t)).ravel()
    col = np.array([1.0, 0.5j, -0.25])
    b = O.from_full(phase[:, None] * col[None], dims, 0)
    lam = m * m + 4 * sum((a * np.sin(q) + bcoef * np.sin(3 * q)) ** 2 for q in p)
    res = O.cg(lat, m, b, 1e-13, 50)
    assert res.status == O.OK and res.iterations <= 2
    np.testing.assert_allclose(res.x, b / lam, atol=1e-12)


def test_cg_status_not_converged_and_breakdown():
    dims = (4, 4, 4, 4)
    w = gen.workload_haar(dims, 22, -1)
    lat = O.lattice_from(w)
    b = w["src"][0]
    r = O.cg(lat, 0.05, b, 1e-14, 3)
    assert r.status == O.NOT_CONVERGED and r.iterations == 3 and r.true_residual > 1e-14
    bad = b.copy()
    bad[0, 0] = np.nan
    r = O.cg(lat, 0.05, bad, 1e-10, 10)
    assert r.status == O.BREAKDOWN


def test_cg_initial_guess_resumes():
    dims = (4, 4, 4, 4)
    w = gen.workload_haar(dims, 23, +1)
    lat = O.lattice_from(w)
    b = w["src"][0]
    r1 = O.cg(lat, 0.1, b, 1e-6, 500)
    r2 = O.cg(lat, 0.1, b, 1e-11, 500, x0=r1.x)
    assert r2.status == O.OK and r2.true_residual <= 1e-11


def test_multishift_reference_dense():
    dims = (4, 4, 4, 4)
    w = gen.workload_haar(dims, 24, -1)
    lat = O.lattice_from(w)
    m = 0.05
    shifts = [0.0, 1e-3, 0.1, 1.0]
    b = w["src"][0]
    M = dense.dense_normal_even(dims, -1, w["fat"], w["naik"], m)
    for s, r in zip(shifts, O.multishift_reference(lat, m, shifts, b, 1e-11, 3000)):
        assert r.status == O.OK
        xd = np.linalg.solve(M + s * np.eye(M.shape[0]), b.ravel())
        assert np.linalg.norm(r.x.ravel() - xd) <= 1e-7 * np.linalg.norm(xd)


def test_quantize_fp16n_format():
    rng = np.random.default_rng(3)
    psi = (rng.standard_normal((5, 3)) + 1j * rng.standard_normal((5, 3))) * 10.0 ** rng.integers(-3, 3, (5, 1))
    q = O.quantize_field_fp16n(psi)
    n = np.maximum(np.abs(psi.real), np.abs(psi.imag)).max(-1, keepdims=True)
    # per site, every component is within half a binary16 ulp of 1 (relative to n)
    assert np.all(np.abs(q - psi) <= (2.0 ** -11 + 2.0 ** -23) * n * np.sqrt(2))
    assert np.all(O.quantize_field_fp16n(np.zeros((2, 3))) == 0)


def test_fp16_format_rounds_once_from_binary64():
    """1 + 2^-11 + 2^-40 is above the binary16 midpoint: one rounding gives
    1 + 2^-10, while rounding through binary32 first would tie down to 1."""
    v = np.array([1 + 2.0 ** -11 + 2.0 ** -40])
    assert O.quantize_links_fp16(v)[0] == 1 + 2.0 ** -10
    psi = np.array([[1 + 2.0 ** -11 + 2.0 ** -40, 0.5, 0.25]], dtype=complex) * 2.0
    q = O.quantize_field_fp16n(psi)
    # the site norm is 2 + 2^-10 + 2^-39 -> binary32 rounds it to 2 + 2^-10
    assert q[0, 0].real == np.float32(2 + 2.0 ** -10)
