"""Pins of the PTC preconditioner oracle: identity, covariance, adjoint, gradients."""
import numpy as np
import pytest

import hisq_inputs as gen
from oracle import hisq as O
from oracle import ptc

DIMS = (4, 4, 4, 6)


@pytest.fixture(scope="module")
def field():
    w = gen.workload_haar(DIMS, 31, -1)
    return w


def test_identity_weights(field):
    b = field["src"][0]
    y, _ = ptc.network_forward(DIMS, -1, field["fat"], ptc.identity_weights(), b)
    np.testing.assert_array_equal(y, b)


@pytest.mark.parametrize("path", range(9))
def test_transport_adjoint(field, path):
    """<chi, T_p psi> = <T_p^+ chi, psi> with T_{+mu}^+ = T_{-mu}."""
    rng = gen.rng_for(31, 11 + path)
    chi = gen.gaussian_full_field(rng, DIMS)
    psi = gen.gaussian_full_field(rng, DIMS)
    X = field["fat"]
    lhs = np.vdot(chi, ptc.transport(DIMS, -1, X, psi, path))
    rhs = np.vdot(ptc.transport(DIMS, -1, X, chi, ptc.adjoint_path(path)), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_transport_matches_dslash_hops(field):
    """Sum of eta-weighted one-hop transports equals the oracle D with W = 0."""
    X = field["fat"]
    nx, ny, nz, nt = DIMS
    psi = gen.gaussian_full_field(gen.rng_for(31, 40), DIMS)
    t, z, y, x = np.meshgrid(*[np.arange(n) for n in (nt, nz, ny, nx)], indexing="ij")
    c = (x, y, z, t)
    acc = np.zeros_like(psi)
    for mu in range(4):
        eta = ((-1.0) ** ((sum(c[:mu]) + 0 * x) % 2))[..., None]
        acc += eta * (ptc.transport(DIMS, -1, X, psi, 1 + 2 * mu)
                      - ptc.transport(DIMS, -1, X, psi, 2 + 2 * mu))
    ref = O.dslash_full(DIMS, -1, X, np.zeros_like(X), psi.reshape(-1, 3)).reshape(psi.shape)
    np.testing.assert_allclose(acc, ref, atol=1e-13)


def test_gauge_covariance(field):
    """N[X^g](g r) = g N[X](r)."""
    X = field["fat"]
    g = gen.gauge_transform(DIMS, gen.rng_for(31, gen.FIELD_GAUGE))
    Xg = np.empty_like(X)
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        Xg[mu] = g @ X[mu] @ np.roll(g, -1, axis=ax).conj().swapaxes(-1, -2)
    ws = ptc.init_weights(np.random.default_rng(5), scale=0.5)
    b = field["src"][0]
    ge = g[ptc.even_mask(DIMS)]
    y, _ = ptc.network_forward(DIMS, -1, X, ws, b)
    yg, _ = ptc.network_forward(DIMS, -1, Xg, ws, np.einsum("sab,sb->sa", ge, b))
    np.testing.assert_allclose(yg, np.einsum("sab,sb->sa", ge, y), atol=1e-12)


def test_weight_gradient_finite_differences(field):
    X = field["fat"]
    rng = np.random.default_rng(9)
    ws = ptc.init_weights(rng, scale=0.5)
    srcs = gen.gaussian_half_field(gen.rng_for(31, 50), DIMS, 2)
    sols = gen.gaussian_half_field(gen.rng_for(31, 51), DIMS, 2)
    lat = O.lattice_from(field)
    A = lambda v: lat.M_e(0.3, v)  # noqa: E731
    L0, gs = ptc.loss_and_grad(DIMS, -1, X, ws, srcs, sols, A)
    h = 1e-6
    for li, (co, ci, p) in [(0, (3, 0, 2)), (1, (5, 2, 7)), (1, (0, 0, 0)), (2, (0, 6, 8))]:
        for part, unit in (("re", 1.0), ("im", 1j)):
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[li][co, ci, p] += h * unit
            wm[li][co, ci, p] -= h * unit
            Lp, _ = ptc.loss_and_grad(DIMS, -1, X, wp, srcs, sols, A)
            Lm, _ = ptc.loss_and_grad(DIMS, -1, X, wm, srcs, sols, A)
            fd = (Lp - Lm) / (2 * h)
            an = gs[li][co, ci, p].real if part == "re" else gs[li][co, ci, p].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (li, co, ci, p, part, fd, an)


def test_input_gradient_is_adjoint(field):
    """<g, J v> = <J^+ g, v> for the (linear) network map J."""
    X = field["fat"]
    ws = ptc.init_weights(np.random.default_rng(2), scale=0.5)
    v = gen.gaussian_half_field(gen.rng_for(31, 60), DIMS)[0]
    g = gen.gaussian_half_field(gen.rng_for(31, 61), DIMS)[0]
    y, acts = ptc.network_forward(DIMS, -1, X, ws, v)
    _, jtg = ptc.network_backward(DIMS, -1, X, ws, acts, g)
    assert abs(np.vdot(g, y) - np.vdot(jtg, v)) < 1e-11 * abs(np.vdot(g, y))


def test_adam_first_step_is_sign_times_lr():
    w = [np.array([[[1.0 + 1.0j]]])]
    g = [np.array([[[0.3 - 2.0j]]])]
    z = [np.zeros_like(w[0])]
    nw, m, v = ptc.adam_step(w, g, z, z, 1, lr=1e-3)
    np.testing.assert_allclose(nw[0], w[0] - 1e-3 * (1 - 1j), atol=1e-9)


def test_adam_three_steps_hand_computed():
    """Three Adam steps with beta1 = beta2 = 1/2 and eps = 0, where every
    moment is a short binary fraction worked out by hand.  The real part sees
    gradients +1, -1, -1 and the imaginary part 2, 2, -2, so a moment that is
    not carried from step to step, a bias correction with the wrong power, or
    real and imaginary moments swapped all change the numbers.
      re: m = 1/2, -1/4, -5/8;  v = 1/2, 3/4, 7/8;  m^ = 1, -1/3, -5/7;  v^ = 1
          w_re = 1 - lr (1 - 1/3 - 5/7) = 1 + lr/21
      im: m = 1, 3/2, -1/4;     v = 2, 3, 7/2;      m^ = 2, 2, -2/7;    v^ = 4
          w_im = 1 - lr (1 + 1 - 1/7) = 1 - 13 lr/7"""
    lr = 0.1
    w = [np.array([[[1.0 + 1.0j]]])]
    m = [np.zeros_like(w[0])]
    v = [np.zeros_like(w[0])]
    for step, g in enumerate((1.0 + 2.0j, -1.0 + 2.0j, -1.0 - 2.0j), start=1):
        w, m, v = ptc.adam_step(w, [np.array([[[g]]])], m, v, step, lr=lr, beta1=0.5, beta2=0.5, eps=0.0)
    assert m[0].ravel()[0] == -0.625 - 0.25j
    assert v[0].ravel()[0] == 0.875 + 3.5j
    np.testing.assert_allclose(w[0].ravel()[0].real, 1.0 + lr / 21, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w[0].ravel()[0].imag, 1.0 - 13 * lr / 7, rtol=0, atol=1e-15)


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the bias-corrected moments are g and g^2 at
    every step, so each step moves each part by lr sign(g) (eps -> 0), with
    the standard decays."""
    w = [np.array([[[0.5 - 0.25j, 2.0 + 0.0j]]])]
    g = [np.array([[[0.3 - 7.0j, -1e-3 + 4.0j]]])]
    m = [np.zeros_like(w[0])]
    v = [np.zeros_like(w[0])]
    lr = 1e-2
    for step in range(1, 6):
        w, m, v = ptc.adam_step(w, g, m, v, step, lr=lr, eps=0.0)
    np.testing.assert_allclose(w[0], np.array([[[0.5 - 0.05 - 0.25j + 0.05j, 2.0 + 0.05 - 0.05j]]]),
                               rtol=0, atol=1e-12)


def test_fcg_identity_preconditioner_is_cg(field):
    lat = O.lattice_from(field)
    b = field["src"][0]
    x, st, it, tr = ptc.fcg(lat, 0.1, b, lambda r: r.copy(), 1e-10, 1000)
    ref = O.cg(lat, 0.1, b, 1e-10, 1000)
    assert st == O.OK and tr <= 1e-10
    assert abs(it - ref.iterations) <= 1


def test_energy_loss_zero_at_exact_inverse_pairs(field):
    """L = 0 when the network output equals x; L = 1 when it outputs zero."""
    lat = O.lattice_from(field)
    A = lambda v: lat.M_e(0.3, v)  # noqa: E731
    x = gen.gaussian_half_field(gen.rng_for(31, 52), DIMS, 1)
    b = np.stack([A(x[0])])
    zero = [np.zeros_like(w) for w in ptc.identity_weights()]
    L, _ = ptc.loss_and_grad(DIMS, -1, field["fat"], zero, b, x, A)
    assert abs(L - 1.0) < 1e-12
    # identity network on b = x (A = identity-like check): e = b - x = 0
    L2, _ = ptc.loss_and_grad(DIMS, -1, field["fat"], ptc.identity_weights(), x, x, A)
    assert L2 == 0.0
