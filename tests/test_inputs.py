"""Pins of the seeded input generators (harness, shared by both paths)."""
import numpy as np

import hisq_inputs as gen


def test_haar_unitary_det_one():
    U = gen.haar_su3(gen.rng_for(0, 1), 2000)
    eye = np.eye(3)
    assert np.abs(U @ U.conj().swapaxes(-1, -2) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


def test_haar_moments():
    """E|tr U|^2 = 1 and E tr U = 0 for Haar SU(3)."""
    U = gen.haar_su3(gen.rng_for(0, 2), 100_000)
    tr = np.trace(U, axis1=-2, axis2=-1)
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 0.03
    assert abs(np.mean(tr)) < 0.02


def test_smooth_links_mean_trace():
    """<Re tr U>/3 = 1 - (2/3) eps^2 + O(eps^4) for U = exp(i eps H)."""
    eps = 0.3
    U = gen.smooth_su3(gen.rng_for(0, 3), 50_000, eps)
    assert np.abs(U @ U.conj().swapaxes(-1, -2) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
    m = np.mean(np.trace(U, axis1=-2, axis2=-1).real) / 3
    # fourth-order term: E tr H^4 / 72 for this normalisation is small at eps = 0.3
    assert abs(m - (1 - 2 / 3 * eps ** 2)) < 0.01


def test_long_links_are_path_products():
    dims = (4, 4, 6, 4)
    v = gen.smooth_links(dims, gen.rng_for(0, 4), 0.3)
    w = gen.long_links_from(v)
    # direction 2 (z), site (x=1, y=2, z=5, t=3): V(z=5) V(z=0) V(z=1)
    ref = v[2, 3, 5, 2, 1] @ v[2, 3, 0, 2, 1] @ v[2, 3, 1, 2, 1]
    np.testing.assert_allclose(w[2, 3, 5, 2, 1], ref, atol=1e-14)


def test_sources_unit_variance_and_seeded():
    a = gen.gaussian_half_field(gen.rng_for(2, 3), (8, 8, 8, 8), 2)
    b = gen.gaussian_half_field(gen.rng_for(2, 3), (8, 8, 8, 8), 2)
    np.testing.assert_array_equal(a, b)
    assert a.shape == (2, 2048, 3)
    assert abs(np.mean(np.abs(a) ** 2) - 1.0) < 0.05


def test_ptc_initial_weights_follow_the_oracle_recipe():
    """The benchmark draws its starting PTC weights from the generator module;
    the draw equals the oracle's initialisation for the same seed."""
    import numpy as np
    from oracle import ptc
    a = gen.ptc_initial_weights(7, 0.2)
    b = ptc.init_weights(np.random.default_rng(7), scale=0.2)
    assert [x.shape for x in a] == [(8, 1, 9), (8, 8, 9), (1, 8, 9)]
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
