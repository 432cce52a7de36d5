"""Link compression on the GPU: the reconstruct-12 check and the W14 format
(fat links in full, Naik links as rows 0 and 1 plus a complex factor z, row 2
rebuilt as z conj(row 0 x row 1)), against the oracle's emulation of the
stored format (oracle/hisq.py quantize_links_w14) on HISQ-smeared links."""
import numpy as np
import pytest
import torch

import hisq_inputs as gen
from oracle import hisq as O
from oracle import smear as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smeared():
    cache = {}

    def get(dims, t_bc, nsrc=1, seed=0):
        key = (dims, t_bc, nsrc, seed)
        if key not in cache:
            U = gen.smooth_links(dims, gen.rng_for(530 + seed, 1), 0.3)
            X, W = S.hisq_smear(U)
            cache[key] = {"dims": dims, "t_bc": t_bc, "fat": np.ascontiguousarray(X),
                          "naik": np.ascontiguousarray(W),
                          "src": gen.gaussian_half_field(gen.rng_for(530 + seed, 2), dims, nsrc),
                          "src_o": gen.gaussian_half_field(gen.rng_for(530 + seed, 3), dims, nsrc)}
        return cache[key]
    return get


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec", ["fp64r12", "fp32r12"])
def test_r12_refuses_smeared_links(gpu_lib, smeared, prec):
    """Neither the HISQ fat link (a sum of paths) nor the Naik link (a real
    multiple of a U(3) matrix) is special unitary: packing them as
    reconstruct-12 is refused."""
    h = gpu_lib
    w = smeared((4, 4, 6, 8), -1)
    lat = h.lattice(w["dims"], w["t_bc"])
    with pytest.raises(h.HisqError) as e:
        h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    assert e.value.status == h.INVALID_ARG
    # one bad link is enough
    su3 = gen.workload_haar(w["dims"], 531, -1)
    fat = su3["fat"].copy()
    fat[2, 1, 0, 1, 3] *= 1.01
    with pytest.raises(h.HisqError):
        h.pack_links_from_host(lat, prec, fat, su3["naik"])
    h.pack_links_from_host(lat, prec, su3["fat"], su3["naik"])   # SU(3): accepted


@pytest.mark.parametrize("prec", ["fp64w14", "fp32w14"])
def test_w14_pack_unpack_matches_the_format(gpu_lib, smeared, prec):
    h = gpu_lib
    w = smeared((4, 4, 6, 8), -1)
    lat = h.lattice(w["dims"], w["t_bc"])
    packed = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    V = int(np.prod(w["dims"]))
    rb = 8 if prec == "fp64w14" else 4
    assert packed.numel() == h.hisq_links_bytes(lat, prec) == 4 * V * (18 + 14) * rb
    f = torch.empty(w["fat"].shape, dtype=torch.complex128, device="cuda")
    n = torch.empty_like(f)
    h.hisq_unpack_links(lat, prec, packed, f, n)
    torch.cuda.synchronize()
    q = O.quantized_lattice(O.Lattice(w["dims"], w["t_bc"], w["fat"], w["naik"]), prec)
    gf, gn = f.cpu().numpy(), n.cpu().numpy()
    np.testing.assert_array_equal(gf, q.X)                   # fat links stored in full
    np.testing.assert_array_equal(gn[..., :2, :], q.W[..., :2, :])
    tol = 1e-16 if prec == "fp64w14" else 2e-8              # row 2 rebuilt in the storage precision
    assert np.abs(gn[..., 2, :] - q.W[..., 2, :]).max() <= tol
    assert np.abs(gn - w["naik"]).max() <= (1e-15 if prec == "fp64w14" else 1e-7)


@pytest.mark.parametrize("prec", ["fp64w14", "fp32w14"])
def test_w14_refuses_naik_links_of_the_wrong_form(gpu_lib, smeared, prec):
    """Fat links passed as the Naik field are not multiples of U(3) matrices."""
    h = gpu_lib
    w = smeared((4, 4, 6, 8), -1)
    lat = h.lattice(w["dims"], w["t_bc"])
    with pytest.raises(h.HisqError) as e:
        h.pack_links_from_host(lat, prec, w["fat"], w["fat"])
    assert e.value.status == h.INVALID_ARG
    # SU(3) links of both kinds fit (z = 1)
    su3 = gen.workload_haar(w["dims"], 532, -1)
    h.pack_links_from_host(lat, prec, su3["fat"], su3["naik"])


@pytest.mark.parametrize("prec", ["fp64w14", "fp32w14"])
@pytest.mark.parametrize("shape", [(0, 1, 128, 1), (1, 1, 64, 1), (0, 2, 64, 2)])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_w14_dslash_on_smeared_links(gpu_lib, smeared, prec, shape, nrhs):
    h = gpu_lib
    dims, t_bc = (6, 4, 8, 10), -1
    w = smeared(dims, t_bc, nrhs)
    lat = h.lattice(dims, t_bc)
    ctx = h.Context(0)
    if shape[3] == 2 and dims[2] % 8:
        shape = (shape[0], shape[1], shape[2], 1)
    h.hisq_set_dslash_shape(lat, prec, nrhs, (shape[0], min(shape[1], nrhs), shape[2], shape[3]), ctx)
    links = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    q = O.quantized_lattice(O.Lattice(dims, t_bc, w["fat"], w["naik"]), prec)
    for parity in (0, 1):
        src = w["src_o"] if parity == 0 else w["src"]
        inp = h.pack_field_from_host(lat, prec, src)
        out = h.empty_field(lat, prec, nrhs)
        h.hisq_dslash(lat, prec, parity, links, inp, out, nrhs, ctx=ctx)
        got = h.unpack_field_to_host(lat, prec, out, nrhs)
        srcq = O.quantize_field(src, prec)
        ref = np.stack([q.D_eo(s) if parity == 0 else q.D_oe(s) for s in srcq])
        tol = 1e-13 if prec == "fp64w14" else 2e-6
        assert relerr(got, ref) <= tol, (parity, relerr(got, ref))
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("lp,fp", [("fp64w14", "fp64"), ("fp32w14", "fp32")])
def test_w14_apply_m_dot(gpu_lib, smeared, lp, fp):
    h = gpu_lib
    dims, t_bc, nrhs, m = (4, 4, 6, 8), 1, 2, 0.1
    w = smeared(dims, t_bc, nrhs)
    lat = h.lattice(dims, t_bc)
    links = h.pack_links_from_host(lat, lp, w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, fp, w["src"])
    out, tmp = h.empty_field(lat, fp, nrhs), h.empty_field(lat, fp, nrhs)
    dots = torch.zeros(nrhs, dtype=torch.float64, device="cuda")
    ws = h.empty_workspace(h.hisq_apply_m_dot_workspace_bytes(lat, nrhs))
    h.hisq_apply_m_dot(lat, lp, fp, m, links, inp, out, tmp, dots, ws, nrhs)
    got = h.unpack_field_to_host(lat, fp, out, nrhs)
    q = O.quantized_lattice(O.Lattice(dims, t_bc, w["fat"], w["naik"]), lp)
    srcq = O.quantize_field(w["src"], fp)
    ref = np.stack([q.M_e(m, s) for s in srcq])
    dref = np.array([np.vdot(a.ravel(), b.ravel()).real for a, b in zip(srcq, ref)])
    tol = 1e-13 if lp == "fp64w14" else 2e-6
    assert relerr(got, ref) <= tol
    assert np.all(np.abs(dots.cpu().numpy() - dref) <= tol * np.abs(dref))


@pytest.mark.parametrize("inner", ["fp64w14", "fp32w14"])
def test_cg_with_w14_inner_links_on_smeared_links(gpu_lib, smeared, inner):
    """Reliable-update CG whose iterations use W14 links, on HISQ-smeared
    links: the oracle's FP64 true residual meets 1e-10."""
    h = gpu_lib
    dims, t_bc, m = (8, 8, 8, 8), -1, 0.05
    w = smeared(dims, t_bc)
    lat = h.lattice(dims, t_bc)
    l64 = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
    lin = h.pack_links_from_host(lat, inner, w["fat"], w["naik"])
    b = h.pack_field_from_host(lat, "fp64", w["src"][0])
    x = h.empty_field(lat, "fp64")
    x.zero_()
    ws = h.empty_workspace(h.hisq_cg_workspace_bytes(lat, inner, 1, 0))
    st, info = h.hisq_cg(lat, m, l64, lin, inner, 1, b, x, 1e-10, 20000, ws)
    assert st == h.OK, info
    sol = h.unpack_field_to_host(lat, "fp64", x)[0]
    res = O.true_residual(O.Lattice(dims, t_bc, w["fat"], w["naik"]), m, w["src"][0], sol)
    print(f"\n{inner}: {info[0]['iterations']} iterations, oracle true residual {res:.2e}")
    assert res <= 1e-10
