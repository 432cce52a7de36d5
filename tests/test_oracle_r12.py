"""Pins of the reconstruct-12 link format (oracle/hisq.py reconstruct12): the
rebuilt third row is the complex conjugate of the cross product of rows 0 and
1, which reproduces exactly the special-unitary matrices and no others."""
import numpy as np

import hisq_inputs as gen
from oracle import hisq as O


def test_special_unitary_matrices_are_reproduced():
    U = gen.haar_su3(gen.rng_for(900, 1), 500)
    np.testing.assert_allclose(O.reconstruct12(U), U, rtol=0, atol=1e-14)
    S = gen.smooth_su3(gen.rng_for(900, 2), 500, 0.3)
    np.testing.assert_allclose(O.reconstruct12(S), S, rtol=0, atol=1e-14)


def test_hand_examples_fix_order_and_conjugation():
    # cyclic permutation (det +1): row 2 comes back
    P = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], dtype=complex)
    np.testing.assert_array_equal(O.reconstruct12(P), P)
    # odd permutation (det -1): row 2 comes back with the opposite sign
    Q = np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1]], dtype=complex)
    np.testing.assert_array_equal(O.reconstruct12(Q)[2], [0, 0, -1])
    # diag(e^ia, e^ib, e^-i(a+b)): only the conjugated cross product gives e^-i(a+b)
    a, b = 0.7, -1.9
    D = np.diag([np.exp(1j * a), np.exp(1j * b), np.exp(-1j * (a + b))])
    np.testing.assert_allclose(O.reconstruct12(D), D, rtol=0, atol=1e-15)
    assert abs(O.reconstruct12(D)[2, 2] - np.exp(1j * (a + b))) > 0.5


def test_u3_phase_is_not_reproduced():
    """A U(3) link e^{i phi} U loses its phase on row 2 (e^{-2 i phi} instead of
    e^{i phi}): the format is only valid for SU(3)."""
    U = gen.haar_su3(gen.rng_for(900, 3), 10)
    phi = 0.4
    V = np.exp(1j * phi) * U
    R = O.reconstruct12(V)
    np.testing.assert_array_equal(R[:, :2], V[:, :2])
    np.testing.assert_allclose(R[:, 2], np.exp(-2j * phi) * U[:, 2], atol=1e-14)
    assert np.abs(R[:, 2] - V[:, 2]).max() > 0.1


def test_r12_lattice_gives_the_same_operator_on_su3_links():
    w = gen.workload_haar((4, 4, 4, 6), 901, -1)
    lat = O.lattice_from(w)
    q = O.quantized_lattice(lat, "fp64r12")
    psi = w["src"][0]
    ref = lat.D_oe(psi)
    assert np.linalg.norm(q.D_oe(psi) - ref) <= 1e-14 * np.linalg.norm(ref)
    q32 = O.quantized_lattice(lat, "fp32r12")
    r32 = O.quantized_lattice(lat, "fp32")
    # rows 0 and 1 as stored in FP32, row 2 rebuilt: close to the FP32-rounded operator
    assert np.linalg.norm(q32.D_oe(psi) - r32.D_oe(psi)) <= 1e-6 * np.linalg.norm(ref)
