"""Pins of the FP64 oracle Dslash against what the mathematics fixes.

Each test checks the oracle against something other than itself: the
free-field closed form (pointwise and the full spectrum), anti-Hermiticity,
gauge covariance, translation by two sites, and the dense matrix assembled
block by block on 4^4.  A dropped term, a wrong sign, a wrong neighbour, a
missing dagger or a transposed link makes at least one of them fail.
"""
import itertools

import numpy as np
import pytest

import hisq_inputs as gen
from oracle import dense
from oracle import hisq as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def unit_links(dims, a):
    nx, ny, nz, nt = dims
    U = np.zeros((4, nt, nz, ny, nx, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = a
    return U


def coords(dims):
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    return [c.ravel() for c in (x, y, z, t)]


def momenta(dims, t_bc):
    """Allowed momenta: 2 pi n / N (periodic), (2n+1) pi / N (antiperiodic time)."""
    axes = []
    for mu, n in enumerate(dims):
        off = 1.0 if (mu == 3 and t_bc == -1) else 0.0
        axes.append([(2 * k + off) * np.pi / n for k in range(n)])
    return list(itertools.product(*axes))


def eta(c, mu):
    return (-1.0) ** (sum(c[:mu]) % 2)


@pytest.mark.parametrize("t_bc", [+1, -1])
@pytest.mark.parametrize("ab", [(1.0, 0.0), (0.0, 1.0), (0.7, -0.3)])
def test_free_field_plane_wave_pointwise(t_bc, ab):
    """(D phi_p)(x) = 2i sum_mu eta_mu(x) [a sin p_mu + b sin 3p_mu] phi_p(x)."""
    a, b = ab
    dims = (4, 6, 4, 8)
    X, W = unit_links(dims, a), unit_links(dims, b)
    c = coords(dims)
    rng = np.random.default_rng(7)
    col = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    moms = momenta(dims, t_bc)
    for p in [moms[i] for i in rng.choice(len(moms), 12, replace=False)]:
        phase = np.exp(1j * sum(pm * cm for pm, cm in zip(p, c)))
        phi = phase[:, None] * col[None, :]
        out = O.dslash_full(dims, t_bc, X, W, phi)
        factor = np.zeros(len(phase), dtype=np.complex128)
        for mu in range(4):
            e = (-1.0) ** (sum(c[:mu]) % 2)
            factor += 2j * e * (a * np.sin(p[mu]) + b * np.sin(3 * p[mu]))
        np.testing.assert_allclose(out, factor[:, None] * phi, atol=1e-12)


@pytest.mark.parametrize("t_bc", [+1, -1])
def test_free_field_spectrum_4x4x4x4(t_bc):
    """Eigenvalues of M_e = m^2 + 4 sum_mu (a sin p_mu + b sin 3 p_mu)^2."""
    dims = (4, 4, 4, 4)
    a, b, m = 1.0, 1.0, 0.1
    X, W = unit_links(dims, a), unit_links(dims, b)
    M = dense.dense_normal_even(dims, t_bc, X, W, m)
    ev = np.sort(np.linalg.eigvalsh(M))
    lam = [m * m + 4 * sum((a * np.sin(p) + b * np.sin(3 * p)) ** 2 for p in pm)
           for pm in momenta(dims, t_bc)]
    # each momentum class {p, p + (pi,pi,pi,pi)} appears twice over all momenta,
    # each with a 3-fold colour degeneracy
    lam = np.sort(np.repeat(lam, 3))[::2]
    np.testing.assert_allclose(ev, lam, atol=1e-12)


@pytest.mark.parametrize("t_bc", [+1, -1])
def test_dense_matches_oracle_and_blocks(t_bc):
    dims = (4, 4, 4, 4)
    w = gen.workload_haar(dims, 11, t_bc)
    D = dense.dense_dslash(dims, t_bc, w["fat"], w["naik"])
    psi = gen.gaussian_full_field(gen.rng_for(11, 9), dims).reshape(-1, 3)
    out = O.dslash_full(dims, t_bc, w["fat"], w["naik"], psi)
    np.testing.assert_allclose(out.ravel(), D @ psi.ravel(), atol=1e-13)
    Dee, Deo, Doe, Doo = dense.parity_blocks(dims, D)
    assert np.abs(Dee).max() == 0 and np.abs(Doo).max() == 0
    # anti-Hermitian: D + D^+ = 0 exactly (entries are sums of the same terms)
    assert np.abs(D + D.conj().T).max() < 1e-14
    # even/odd blocks agree with the oracle's even/odd application
    po = O.from_full(psi, dims, 1)
    np.testing.assert_allclose(O.dslash(dims, t_bc, w["fat"], w["naik"], po, 0).ravel(),
                               Deo @ po.ravel(), atol=1e-13)
    # M_e is Hermitian with spectrum >= m^2
    m = 0.1
    M = m * m * np.eye(Deo.shape[0]) - Deo @ Doe
    assert np.abs(M - M.conj().T).max() < 1e-12
    assert np.linalg.eigvalsh(M).min() >= m * m - 1e-12


@pytest.mark.parametrize("dims,t_bc", [((8, 8, 8, 8), +1), ((8, 8, 8, 8), -1),
                                      ((4, 6, 8, 6), -1)])
def test_anti_hermiticity(dims, t_bc):
    """<chi_e, D_eo psi_o> = -<D_oe chi_e, psi_o>."""
    w = gen.workload_haar(dims, 12, t_bc)
    lat = O.lattice_from(w)
    chi = gen.gaussian_half_field(gen.rng_for(12, 7), dims)[0]
    psi = gen.gaussian_half_field(gen.rng_for(12, 8), dims)[0]
    lhs = O.vdot(chi, lat.D_eo(psi))
    rhs = -O.vdot(lat.D_oe(chi), psi)
    scale = O.norm(chi) * O.norm(lat.D_eo(psi))
    assert abs(lhs - rhs) <= 1e-14 * scale


def _shift(a, mu, k):
    """a(x + k mu) for arrays indexed (.., Nt, Nz, Ny, Nx, ...) starting at axis 0."""
    ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
    return np.roll(a, -k, axis=ax)


@pytest.mark.parametrize("t_bc", [+1, -1])
def test_gauge_covariance(t_bc):
    """D[X^g] (g psi) = g D[X] psi with X^g_mu(x) = g(x) X_mu(x) g(x+mu)^+."""
    dims = (6, 4, 4, 8)
    w = gen.workload_haar(dims, 13, t_bc)
    g = gen.gauge_transform(dims, gen.rng_for(13, gen.FIELD_GAUGE))
    Xg = np.empty_like(w["fat"])
    Wg = np.empty_like(w["naik"])
    for mu in range(4):
        gd1 = _shift(g, mu, 1).conj().swapaxes(-1, -2)
        gd3 = _shift(g, mu, 3).conj().swapaxes(-1, -2)
        Xg[mu] = g @ w["fat"][mu] @ gd1
        Wg[mu] = g @ w["naik"][mu] @ gd3
    psi = gen.gaussian_full_field(gen.rng_for(13, 9), dims)
    gpsi = np.einsum("...ab,...b->...a", g, psi)
    lhs = O.dslash_full(dims, t_bc, Xg, Wg, gpsi.reshape(-1, 3)).reshape(psi.shape)
    rhs = np.einsum("...ab,...b->...a", g,
                    O.dslash_full(dims, t_bc, w["fat"], w["naik"], psi.reshape(-1, 3)).reshape(psi.shape))
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


@pytest.mark.parametrize("mu", [0, 1, 2, 3])
@pytest.mark.parametrize("t_bc", [+1, -1])
def test_translation_by_two_sites(mu, t_bc):
    """Shifting every field by two sites commutes with D (eta is 2-periodic)."""
    dims = (6, 4, 8, 6)
    w = gen.workload_haar(dims, 14, t_bc)
    psi = gen.gaussian_full_field(gen.rng_for(14, 9), dims)

    def shift_field(f):
        s = _shift(f, mu, 2)
        if mu == 3:       # the two slices that wrapped carry the time boundary sign
            s = s.copy()
            s[-2:] *= t_bc
        return s

    Xs = np.stack([_shift(w["fat"][nu], mu, 2) for nu in range(4)])
    Ws = np.stack([_shift(w["naik"][nu], mu, 2) for nu in range(4)])
    lhs = O.dslash_full(dims, t_bc, Xs, Ws, shift_field(psi).reshape(-1, 3)).reshape(psi.shape)
    rhs = shift_field(O.dslash_full(dims, t_bc, w["fat"], w["naik"],
                                    psi.reshape(-1, 3)).reshape(psi.shape))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_naive_staggered_special_case():
    """W = 0 leaves the textbook naive staggered operator: free M_e = m^2 + 4 sum sin^2 p."""
    dims = (4, 4, 4, 4)
    X, W = unit_links(dims, 1.0), unit_links(dims, 0.0)
    m = 0.3
    ev = np.sort(np.linalg.eigvalsh(dense.dense_normal_even(dims, -1, X, W, m)))
    lam = np.sort(np.repeat([m * m + 4 * sum(np.sin(p) ** 2 for p in pm)
                             for pm in momenta(dims, -1)], 3))[::2]
    np.testing.assert_allclose(ev, lam, atol=1e-12)


def test_site_spot_check_matches_full():
    dims = (8, 4, 4, 6)
    w = gen.workload_haar(dims, 15, -1)
    psi_o = gen.gaussian_half_field(gen.rng_for(15, 3), dims)[0]
    full = O.dslash(dims, -1, w["fat"], w["naik"], psi_o, 0)
    ev_sites = O.parity_sites(dims, 0)
    pick = np.array([0, 5, 17, len(ev_sites) - 1])
    spot = O.dslash_at(dims, -1, w["fat"], w["naik"], psi_o, 1, ev_sites[pick])
    np.testing.assert_array_equal(spot, full[pick])


def test_invalid_extents():
    with pytest.raises(ValueError):
        O.dslash_full((0, 4, 4, 4), 1, np.zeros((4, 0, 3, 3)), np.zeros((4, 0, 3, 3)),
                      np.zeros((0, 3)))
