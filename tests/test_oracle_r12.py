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


# ---------------------------------------------------------------------------
# The 14-real Naik-link format: rows 0 and 1 plus one complex factor z, row 2
# rebuilt as z conj(row0 x row1).
# ---------------------------------------------------------------------------

def test_w14_factor_is_one_for_su3_and_the_determinant_for_u3():
    U = gen.haar_su3(gen.rng_for(902, 1), 200)
    np.testing.assert_allclose(O.scaled_row2_factor(U), 1.0, rtol=0, atol=1e-14)
    phi = gen.rng_for(902, 2).uniform(-np.pi, np.pi, 200)
    V = np.exp(1j * phi)[:, None, None] * U            # U(3), det V = e^{3 i phi}
    z = O.scaled_row2_factor(V)
    np.testing.assert_allclose(z, np.linalg.det(V), rtol=0, atol=1e-13)
    np.testing.assert_allclose(z, np.exp(3j * phi), rtol=0, atol=1e-13)
    np.testing.assert_allclose(O.reconstruct_scaled(V, z), V, rtol=0, atol=1e-14)


def test_w14_reproduces_real_multiples_of_u3():
    """a V with V in U(3): z = det V / a, and the rebuilt matrix is a V."""
    U = gen.haar_su3(gen.rng_for(902, 3), 50)
    V = np.exp(0.3j) * U
    a = -1.0 / 24.0
    W = a * V
    z = O.scaled_row2_factor(W)
    np.testing.assert_allclose(z, np.linalg.det(V) / a, rtol=1e-13, atol=0)
    np.testing.assert_allclose(O.reconstruct_scaled(W, z), W, rtol=0, atol=1e-15)


def test_w14_hand_example():
    """diag(2, 3, 5): c = conj(row0 x row1) = (0, 0, 6), so z = 5/6 exactly."""
    D = np.diag([2.0, 3.0, 5.0]).astype(complex)
    assert O.scaled_row2_factor(D) == 5.0 / 6.0
    np.testing.assert_allclose(O.reconstruct_scaled(D, O.scaled_row2_factor(D)), D, rtol=1e-15)
    # a row 2 with a component off the cross product is not reproduced
    E = D.copy()
    E[2, 0] = 1.0
    R = O.reconstruct_scaled(E, O.scaled_row2_factor(E))
    assert abs(R[2, 0] - 1.0) == 1.0


def test_w14_reproduces_hisq_naik_links_but_r12_does_not():
    """The smeared Naik link c_Naik Y(x) Y(x+mu) Y(x+2mu) with Y in U(3) is a
    real multiple of a U(3) matrix: W14 keeps it, reconstruct-12 does not, and
    the fat link X (a sum of paths) fits neither."""
    from oracle import smear as S
    dims = (4, 4, 4, 4)
    U = gen.smooth_links(dims, gen.rng_for(903, 1), 0.3)
    X, W = S.hisq_smear(U)
    W = np.asarray(W).reshape(-1, 3, 3)
    X = np.asarray(X).reshape(-1, 3, 3)
    Wq = O.quantize_links_w14(W, "fp64")
    assert np.abs(Wq - W).max() <= 1e-13 * np.abs(W).max()
    assert np.abs(O.reconstruct12(W) - W).max() > 1e-3 * np.abs(W).max()
    Xq = O.reconstruct_scaled(X, O.scaled_row2_factor(X))
    assert np.abs(Xq - X).max() > 1e-6 * np.abs(X).max()


def test_w14_lattice_on_smeared_links_gives_the_same_operator():
    from oracle import smear as S
    dims, t_bc = (4, 4, 4, 6), -1
    U = gen.smooth_links(dims, gen.rng_for(904, 1), 0.3)
    X, W = S.hisq_smear(U)
    lat = O.Lattice(dims, t_bc, np.asarray(X), np.asarray(W))
    psi = gen.gaussian_half_field(gen.rng_for(904, 2), dims)[0]
    ref = lat.D_oe(psi)
    q = O.quantized_lattice(lat, "fp64w14")
    assert np.linalg.norm(q.D_oe(psi) - ref) <= 1e-13 * np.linalg.norm(ref)
    q32 = O.quantized_lattice(lat, "fp32w14")
    r32 = O.quantized_lattice(lat, "fp32")
    assert np.linalg.norm(q32.D_oe(psi) - r32.D_oe(psi)) <= 1e-6 * np.linalg.norm(ref)
    # reconstruct-12 of the same links is a different operator
    q12 = O.quantized_lattice(lat, "fp64r12")
    assert np.linalg.norm(q12.D_oe(psi) - ref) > 1e-3 * np.linalg.norm(ref)
