"""Pins of the chiral-condensate oracle (oracle/condensate.py): the even-odd
reduction (1/V) Tr (D + m)^-1 = (2 m / V) Tr_e M_e^-1, the free-field closed
form, and the stochastic estimator against both."""
import numpy as np
import pytest

import hisq_inputs as gen
from oracle import condensate as C
from oracle import dense
from oracle import hisq as O


def unit_links(dims, a):
    V = int(np.prod(dims))
    return np.broadcast_to(a * np.eye(3, dtype=np.complex128), (4, V, 3, 3)).reshape(
        (4,) + tuple(reversed(dims)) + (3, 3)).copy()


@pytest.mark.parametrize("t_bc", [+1, -1])
def test_even_odd_reduction_of_the_trace(t_bc):
    dims = (4, 4, 4, 4)
    w = gen.workload_haar(dims, 70, t_bc)
    for m in (0.05, 0.3):
        full = C.exact_dense(dims, t_bc, w["fat"], w["naik"], m)
        even = C.exact_even(dims, t_bc, w["fat"], w["naik"], m)
        assert abs(full - even) <= 1e-12 * abs(full)
        assert full > 0


@pytest.mark.parametrize("t_bc", [+1, -1])
@pytest.mark.parametrize("ab", [(1.0, 0.0), (1.0, 0.5), (0.3, -0.8)])
def test_free_field_closed_form(t_bc, ab):
    dims = (4, 4, 4, 4)
    a, b = ab
    X, W = unit_links(dims, a), unit_links(dims, b)
    m = 0.2
    assert abs(C.free_field(dims, t_bc, a, b, m) - C.exact_dense(dims, t_bc, X, W, m)) <= 1e-12
    # heavy-mass limit: (D + m)^-1 -> 1/m, so pbp -> 3/m
    assert abs(C.free_field(dims, t_bc, a, b, 1e4) * 1e4 / 3 - 1) < 1e-6


def test_samples_are_the_quadratic_forms():
    dims = (4, 4, 4, 6)
    w = gen.workload_haar(dims, 71, -1)
    lat = O.lattice_from(w)
    m = 0.1
    noise = gen.gaussian_half_field(gen.rng_for(71, 40), dims, 3)
    M = dense.dense_normal_even(dims, -1, w["fat"], w["naik"], m)
    V = int(np.prod(dims))
    ref = [2 * m * np.vdot(e.ravel(), np.linalg.solve(M, e.ravel())).real / V for e in noise]
    np.testing.assert_allclose(C.samples(lat, m, noise), ref, rtol=1e-9)


def test_estimator_converges_to_the_trace():
    dims = (4, 4, 4, 4)
    w = gen.workload_haar(dims, 72, -1)
    lat = O.lattice_from(w)
    m = 0.2
    noise = gen.gaussian_half_field(gen.rng_for(72, 41), dims, 200)
    mean, err = C.estimate(C.samples(lat, m, noise, tol=1e-10))
    exact = C.exact_even(dims, -1, w["fat"], w["naik"], m)
    assert abs(mean - exact) <= 4 * err
    assert err < 0.1 * exact
