"""GPU HISQ link smearing against the oracle (oracle/smear.py), FP64.

The GPU projects to U(3) with the closed-form inverse square root of V^+ V
(eigenvalues from the characteristic cubic); the oracle uses an eigen-
decomposition.  Both are backward stable, so the difference scales with the
conditioning of V^+ V: 1e-12 relative on smooth links, 1e-10 on Haar-random
thin links (whose level-1 links are far from unitary), printed with the
smallest singular value seen."""
import numpy as np
import pytest
import torch

import hisq_inputs as gen
from oracle import hisq as O
from oracle import smear as S

pytestmark = pytest.mark.gpu


def run(h, dims, U, eps=0.0):
    lat = h.lattice(dims, -1)
    thin = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    fat, naik = torch.empty_like(thin), torch.empty_like(thin)
    ws = h.empty_workspace(h.hisq_smear_workspace_bytes(lat))
    h.hisq_smear_links(lat, thin, fat, naik, ws, eps)
    torch.cuda.synchronize()
    return lat, fat.cpu().numpy(), naik.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("kind,dims,tol", [("smooth", (4, 4, 4, 4), 1e-12), ("smooth", (6, 4, 8, 4), 1e-12),
                                           ("haar", (4, 4, 4, 6), 1e-10)])
def test_smear_matches_oracle(gpu_lib, kind, dims, tol):
    h = gpu_lib
    rng = gen.rng_for(520, 1)
    U = gen.smooth_links(dims, rng, 0.6) if kind == "smooth" else gen.haar_links(dims, rng)
    _, X, W = run(h, dims, U, eps=0.1)
    Xr, Wr = S.hisq_smear(U, eps=0.1)
    V = S.smear_level(U, **S.LEVEL1)
    smin = np.sqrt(np.linalg.eigvalsh(np.conj(np.swapaxes(V, -1, -2)) @ V).min())
    print(f"\n{kind} {dims}: X {rel(X, Xr):.2e} W {rel(W, Wr):.2e} (smallest singular value of V {smin:.3f})")
    assert rel(X, Xr) <= tol and rel(W, Wr) <= tol


def test_unit_links_give_the_coefficient_sums(gpu_lib):
    h = gpu_lib
    dims = (4, 4, 4, 4)
    nx, ny, nz, nt = dims
    U = np.zeros((4, nt, nz, ny, nx, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    _, X, W = run(h, dims, U)
    np.testing.assert_allclose(X, U * 9 / 8, atol=1e-15)
    np.testing.assert_allclose(W, -U / 24, atol=1e-15)


def test_smeared_links_drive_the_dslash(gpu_lib):
    """Smear on the GPU, pack, apply D_oe: equals the oracle's Dslash with the
    oracle's smeared links."""
    h = gpu_lib
    dims = (4, 4, 6, 8)
    U = gen.smooth_links(dims, gen.rng_for(521, 1), 0.4)
    lat, X, W = run(h, dims, U)
    Xr, Wr = S.hisq_smear(U)
    links = h.pack_links_from_host(lat, "fp64", X, W)
    src = gen.gaussian_half_field(gen.rng_for(521, 3), dims)[0]
    inp = h.pack_field_from_host(lat, "fp64", src)
    out = h.empty_field(lat, "fp64")
    h.hisq_dslash(lat, "fp64", 1, links, inp, out)
    got = h.unpack_field_to_host(lat, "fp64", out)[0]
    ref = O.dslash(dims, -1, Xr, Wr, src, 1)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
