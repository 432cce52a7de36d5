"""Pins of the HISQ smearing oracle (oracle/smear.py): nested staples against
explicit path products, unit links, gauge covariance, and the U(3) projection
against the polar decomposition of a library routine."""
import numpy as np
import pytest
import scipy.linalg

import hisq_inputs as gen
from oracle import smear as S


def unit(dims, c=1.0):
    nx, ny, nz, nt = dims
    U = np.zeros((4, nt, nz, ny, nx, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = c
    return U


@pytest.mark.parametrize("level", ["LEVEL1", "LEVEL2"])
def test_nested_staples_equal_path_products(level):
    dims = (4, 4, 6, 4)
    U = gen.haar_links(dims, gen.rng_for(510, 1))
    co = getattr(S, level)
    F = S.smear_level(U, **co)
    for x in [(0, 0, 0, 0), (3, 1, 5, 2), (2, 3, 1, 3)]:
        for mu in range(4):
            ref = S.path_sum_at(U, dims, x, mu, **co)
            assert np.abs(F[mu, x[3], x[2], x[1], x[0]] - ref).max() < 1e-14


def test_path_counts_on_unit_links():
    """Unit links: every path is 1, so the levels give the coefficient sums
    c1 + 6 c3 + 24 c5 + 48 c7 (+ 6 c_Lepage): 1 and 9/8; the Naik link -1/24."""
    dims = (4, 4, 4, 4)
    X, W = S.hisq_smear(unit(dims))
    np.testing.assert_allclose(X, unit(dims, 9 / 8), atol=1e-15)
    np.testing.assert_allclose(W, unit(dims, -1 / 24), atol=1e-15)
    np.testing.assert_allclose(S.smear_level(unit(dims), **S.LEVEL1), unit(dims), atol=1e-15)
    # the free dispersion 9/8 sin p - 1/24 sin 3p has no p^3 term (Naik improvement)
    p = 1e-2
    assert abs(9 / 8 * np.sin(p) - np.sin(3 * p) / 24 - p) < 1e-9


def test_gauge_covariance():
    dims = (4, 4, 4, 6)
    U = gen.smooth_links(dims, gen.rng_for(511, 1), 0.5)
    g = gen.gauge_transform(dims, gen.rng_for(511, 5))
    def transform(L, k):
        out = np.empty_like(L)
        for mu in range(4):
            out[mu] = g @ L[mu] @ np.conj(np.swapaxes(np.roll(g, -k, axis=S.AXIS[mu]), -1, -2))
        return out
    X, W = S.hisq_smear(U)
    Xg, Wg = S.hisq_smear(transform(U, 1))
    np.testing.assert_allclose(Xg, transform(X, 1), atol=1e-13)
    np.testing.assert_allclose(Wg, transform(W, 3), atol=1e-13)


def test_projection_is_the_polar_factor():
    rng = gen.rng_for(512, 1)
    V = rng.standard_normal((50, 3, 3)) + 1j * rng.standard_normal((50, 3, 3))
    Y = S.u3_project(V)
    for k in range(50):
        np.testing.assert_allclose(Y[k], scipy.linalg.polar(V[k])[0], atol=1e-13)
    np.testing.assert_allclose(np.conj(np.swapaxes(Y, -1, -2)) @ Y, np.broadcast_to(np.eye(3), Y.shape), atol=1e-13)
    U = gen.haar_su3(gen.rng_for(512, 2), 20)
    np.testing.assert_allclose(S.u3_project(2.5 * U), U, atol=1e-14)
