"""GPU parity of the packed layouts, the Dslash and M_e against the FP64 oracle.

Tolerances:
  FP64       relative L2 and max-norm error <= 1e-13 against the oracle.
  FP32       against the oracle evaluated in FP64 on FP32-rounded inputs
             (same storage rounding as the kernel): relative <= 1e-6, which
             bounds the FP32 accumulation error of 16 mat-vecs.
  FP16N      against the oracle on inputs rounded to the FP16+norm format; the
             output is itself rounded to that format, so each component may
             differ by half a binary16 ulp of its site norm (2^-12 n) plus the
             FP32 accumulation error.
  R12        reconstruct-12 links (rows 0 and 1 stored, row 2 rebuilt on the
             GPU in the storage precision): FP64R12 <= 1e-13 against the oracle
             on the original SU(3) links; FP32R12 <= 1e-6 against the oracle
             on the FP32-rounded rows with row 2 rebuilt in FP64.
"""
import numpy as np
import pytest
import torch

import hisq_inputs as gen
from oracle import hisq as O

pytestmark = pytest.mark.gpu

LATTICES = [((4, 4, 4, 4), +1), ((8, 8, 8, 8), +1), ((8, 8, 8, 8), -1), ((6, 4, 8, 10), -1),
            ((12, 12, 12, 4), -1)]


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def fields():
    cache = {}

    def get(dims, t_bc, nsrc=1, kind="haar"):
        key = (dims, t_bc, nsrc, kind)
        if key not in cache:
            k = 100 + len(cache)
            if kind == "haar":
                w = gen.workload_haar(dims, k, t_bc, nsrc)
            else:
                w = gen.workload_smooth(dims, k, t_bc, 0.3, nsrc)
            w["src_o"] = gen.gaussian_half_field(gen.rng_for(k, 20), dims, nsrc)
            cache[key] = w
        return cache[key]
    return get


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16n"])
def test_pack_unpack_field_format(gpu_lib, fields, prec):
    h = gpu_lib
    w = fields((6, 4, 8, 10), -1, 3)
    lat = h.lattice(w["dims"], w["t_bc"])
    src = w["src"] * np.array([1.0, 1e-3, 37.0])[:, None, None]
    src[1, 5] = 0.0                      # a zero site keeps a zero norm
    packed = h.pack_field_from_host(lat, prec, src)
    back = h.unpack_field_to_host(lat, prec, packed, 3)
    # bit-exact agreement with the storage format as the oracle defines it
    np.testing.assert_array_equal(back, O.quantize_field(src, prec))


@pytest.mark.parametrize("nrhs", [1, 2, 3, 4, 5])
def test_fp32_field_pair_layout(gpu_lib, fields, nrhs):
    """The packed FP32 layout as the header states it, written out here from
    that description: one column is [colour][site] of {re, im}; in a field of
    several columns, columns 2j and 2j + 1 share 16-byte records
    {re, im of 2j, re, im of 2j + 1}, [pair][colour][site], the second slot
    of the last pair unused for an odd number of columns."""
    h = gpu_lib
    w = fields((6, 4, 8, 10), -1, 5)
    lat = h.lattice(w["dims"], w["t_bc"])
    src = w["src"][:nrhs]
    vh = src.shape[1]
    cols = nrhs + (nrhs % 2) if nrhs >= 2 else 1
    assert h.hisq_field_bytes(lat, "fp32", nrhs) == cols * vh * 24
    raw = h.pack_field_from_host(lat, "fp32", src).view(torch.float32).cpu().numpy()
    q = src.astype(np.complex64)
    if nrhs == 1:
        want = np.stack([q[0].real.T, q[0].imag.T], axis=-1).reshape(-1)   # [colour][site][re, im]
        np.testing.assert_array_equal(raw, want)
        return
    rec = raw.reshape(cols // 2, 3, vh, 4)                                  # [pair][colour][site][4]
    for r in range(nrhs):
        np.testing.assert_array_equal(rec[r // 2, :, :, 2 * (r % 2)], q[r].real.T)
        np.testing.assert_array_equal(rec[r // 2, :, :, 2 * (r % 2) + 1], q[r].imag.T)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16n"])
def test_pack_unpack_links_format(gpu_lib, fields, prec):
    h = gpu_lib
    w = fields((6, 4, 8, 10), -1, 1, "smooth")
    lat = h.lattice(w["dims"], w["t_bc"])
    packed = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    f = torch.empty(w["fat"].shape, dtype=torch.complex128, device="cuda")
    n = torch.empty_like(f)
    h.hisq_unpack_links(lat, prec, packed, f, n)
    torch.cuda.synchronize()
    ql = O.quantized_lattice(O.lattice_from(w), prec)
    np.testing.assert_array_equal(f.cpu().numpy(), ql.X)
    np.testing.assert_array_equal(n.cpu().numpy(), ql.W)


@pytest.mark.parametrize("prec", ["fp64r12", "fp32r12"])
def test_pack_unpack_links_r12(gpu_lib, fields, prec):
    """Rows 0 and 1 come back exactly as stored; row 2 is rebuilt from them."""
    h = gpu_lib
    w = fields((6, 4, 8, 10), -1, 1, "smooth")
    lat = h.lattice(w["dims"], w["t_bc"])
    packed = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    assert packed.numel() * 3 == h.hisq_links_bytes(lat, prec[:4]) * 2
    f = torch.empty(w["fat"].shape, dtype=torch.complex128, device="cuda")
    n = torch.empty_like(f)
    h.hisq_unpack_links(lat, prec, packed, f, n)
    torch.cuda.synchronize()
    ql = O.quantized_lattice(O.lattice_from(w), prec)
    tol = 1e-15 if prec == "fp64r12" else 1e-6
    for got, ref, orig in ((f.cpu().numpy(), ql.X, w["fat"]), (n.cpu().numpy(), ql.W, w["naik"])):
        np.testing.assert_array_equal(got[..., :2, :], ref[..., :2, :])
        assert np.abs(got[..., 2, :] - ref[..., 2, :]).max() <= tol
        assert np.abs(got - orig).max() <= (1e-14 if prec == "fp64r12" else 1e-6)


@pytest.mark.parametrize("prec", ["fp64r12", "fp32r12"])
@pytest.mark.parametrize("dims,t_bc", [((8, 8, 8, 8), -1), ((6, 4, 8, 10), +1), ((12, 12, 12, 4), -1)])
def test_dslash_r12(gpu_lib, fields, prec, dims, t_bc):
    h = gpu_lib
    w = fields(dims, t_bc)
    lat = h.lattice(dims, t_bc)
    lat_o = O.lattice_from(w)
    lat_q = O.quantized_lattice(lat_o, prec)
    links = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    for parity in (0, 1):
        src = w["src_o"][0] if parity == 0 else w["src"][0]
        inp = h.pack_field_from_host(lat, prec, src)
        out = h.empty_field(lat, prec)
        h.hisq_dslash(lat, prec, parity, links, inp, out)
        got = h.unpack_field_to_host(lat, prec, out)[0]
        if prec == "fp64r12":
            ref = lat_o.D_eo(src) if parity == 0 else lat_o.D_oe(src)
            assert relerr(got, ref) <= 1e-13
            assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
        else:
            srcq = O.quantize_field(src, prec)
            ref = lat_q.D_eo(srcq) if parity == 0 else lat_q.D_oe(srcq)
            assert relerr(got, ref) <= 1e-6


@pytest.mark.parametrize("dims,t_bc", LATTICES)
@pytest.mark.parametrize("parity", [0, 1])
def test_dslash_fp64(gpu_lib, fields, dims, t_bc, parity):
    h = gpu_lib
    w = fields(dims, t_bc)
    lat = h.lattice(dims, t_bc)
    lat_o = O.lattice_from(w)
    links = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
    src = w["src_o"][0] if parity == 0 else w["src"][0]
    inp = h.pack_field_from_host(lat, "fp64", src)
    out = h.empty_field(lat, "fp64")
    h.hisq_dslash(lat, "fp64", parity, links, inp, out)
    got = h.unpack_field_to_host(lat, "fp64", out)[0]
    ref = lat_o.D_eo(src) if parity == 0 else lat_o.D_oe(src)
    assert relerr(got, ref) <= 1e-13
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("fp16n", None)])
@pytest.mark.parametrize("dims,t_bc", [((8, 8, 8, 8), -1), ((6, 4, 8, 10), +1)])
def test_dslash_reduced_precision(gpu_lib, fields, prec, tol, dims, t_bc):
    h = gpu_lib
    w = fields(dims, t_bc, kind="smooth")
    lat = h.lattice(dims, t_bc)
    lat_q = O.quantized_lattice(O.lattice_from(w), prec)
    links = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    for parity in (0, 1):
        src = w["src_o"][0] if parity == 0 else w["src"][0]
        inp = h.pack_field_from_host(lat, prec, src)
        out = h.empty_field(lat, prec)
        h.hisq_dslash(lat, prec, parity, links, inp, out)
        got = h.unpack_field_to_host(lat, prec, out)[0]
        srcq = O.quantize_field(src, prec)
        ref = lat_q.D_eo(srcq) if parity == 0 else lat_q.D_oe(srcq)
        if prec == "fp32":
            assert relerr(got, ref) <= tol
        else:
            n = np.maximum(np.abs(ref.real), np.abs(ref.imag)).max(-1, keepdims=True)
            bound = (2.0 ** -12 + 2e-6) * n + 1e-6 * np.abs(ref).max()
            err = np.maximum(np.abs(got.real - ref.real), np.abs(got.imag - ref.imag))
            worst = np.unravel_index(np.argmax(err / bound), err.shape)
            assert np.all(err <= bound), (
                f"parity {parity} site {worst[0]} colour {worst[1]}: err {err[worst]:.3e} "
                f"bound {bound[worst[0], 0]:.3e} n {n[worst[0], 0]:.3e} got {got[worst]} ref {ref[worst]} "
                f"sites over: {int((err > bound).any(-1).sum())}")
        # storage error vs the exact FP64 operator stays at the format's level
        ref64 = O.lattice_from(w).D_eo(src) if parity == 0 else O.lattice_from(w).D_oe(src)
        assert relerr(got, ref64) <= (1e-6 if prec == "fp32" else 4e-3)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16n"])
@pytest.mark.parametrize("nrhs", [3, 16])
@pytest.mark.parametrize("variant", [0, 1])
def test_dslash_multi_rhs_columns(gpu_lib, fields, prec, nrhs, variant):
    """Each column of the batched Dslash equals, bit for bit, the single-RHS
    Dslash with the same thread mapping (same summation order)."""
    h = gpu_lib
    dims, t_bc = (8, 4, 6, 8), -1
    w = fields(dims, t_bc, nrhs)
    lat = h.lattice(dims, t_bc)
    ctx = h.Context(0)
    h.hisq_set_dslash_shape(lat, prec, nrhs, (variant, 8 if prec != "fp64" else 4, 256, 1), ctx)
    h.hisq_set_dslash_shape(lat, prec, 1, (variant, 1, 256, 1), ctx)
    links = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, prec, w["src_o"])
    out = h.empty_field(lat, prec, nrhs)
    h.hisq_dslash(lat, prec, 0, links, inp, out, nrhs, ctx=ctx)
    got = h.unpack_field_to_host(lat, prec, out, nrhs)
    for r in range(nrhs):
        one_in = h.pack_field_from_host(lat, prec, w["src_o"][r])
        one_out = h.empty_field(lat, prec)
        h.hisq_dslash(lat, prec, 0, links, one_in, one_out, 1, ctx=ctx)
        one = h.unpack_field_to_host(lat, prec, one_out)[0]
        np.testing.assert_array_equal(got[r], one)
    if prec == "fp64":
        ref = O.lattice_from(w).D_eo(w["src_o"])
        assert relerr(got, ref) <= 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp64r12", "fp32r12"])
def test_apply_m(gpu_lib, fields, prec):
    h = gpu_lib
    dims, t_bc = (8, 8, 8, 8), -1
    w = fields(dims, t_bc, 2)
    lat = h.lattice(dims, t_bc)
    links = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, prec, w["src"])
    out = h.empty_field(lat, prec, 2)
    tmp = h.empty_field(lat, prec, 2)
    h.hisq_apply_m(lat, prec, 0.1, links, inp, out, tmp, 2)
    got = h.unpack_field_to_host(lat, prec, out, 2)
    lat_q = O.quantized_lattice(O.lattice_from(w), prec)
    ref = np.stack([lat_q.M_e(0.1, O.quantize_field(s, prec)) for s in w["src"]])
    assert relerr(got, ref) <= (1e-13 if prec.startswith("fp64") else 2e-6)


# (link precision, field precision) pairs of the operators the solvers iterate
# with; FP16N links with FP32 fields is the inner operator of FP16N CG.
M_DOT_PAIRS = [("fp64", "fp64"), ("fp32", "fp32"), ("fp16n", "fp32"), ("fp64r12", "fp64"), ("fp32r12", "fp32")]


def _m_dot_reference(w, lp, fp, mass, src):
    """Oracle M_e on the stored links and the stored input (FP64 arithmetic)."""
    lat_q = O.quantized_lattice(O.lattice_from(w), lp)
    srcq = O.quantize_field(src, fp)
    ref = np.stack([lat_q.M_e(mass, s) for s in srcq])
    dots = np.array([np.vdot(a.ravel(), b.ravel()).real for a, b in zip(srcq, ref)])
    return ref, dots


def _check_m_dot(got, dots, ref, dref, lp, what):
    """Element-wise bound: every component within tol * max|ref| (L2 within
    tol too); the fused <in, M_e in> within tol relative (a sum of positive
    terms m^2 |p|^2 + |D_oe p|^2, no cancellation)."""
    tol = 1e-13 if lp.startswith("fp64") else 2e-6
    err = np.abs(got - ref)
    bound = tol * np.abs(ref).max()
    assert err.max() <= bound, (what, float(err.max()), bound)
    assert relerr(got, ref) <= tol, what
    assert np.all(np.abs(dots - dref) <= tol * np.abs(dref)), (what, dots, dref)


@pytest.mark.parametrize("lp,fp", M_DOT_PAIRS)
@pytest.mark.parametrize("variant", [0, 1])
def test_apply_m_dot_matches_oracle(gpu_lib, fields, lp, fp, variant):
    """M_e and the fused Re <p, M_e p> of every solver operator, both thread
    mappings, 3 right-hand sides on a lattice with a ragged tail."""
    h = gpu_lib
    dims, t_bc, nrhs, mass = (6, 4, 8, 10), -1, 3, 0.1
    w = fields(dims, t_bc, nrhs, "smooth")
    lat = h.lattice(dims, t_bc)
    ctx = h.Context(0)
    h.hisq_set_dslash_shape(lat, lp, nrhs, (variant, 2, 128, 1), ctx)
    links = h.pack_links_from_host(lat, lp, w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, fp, w["src"])
    out, tmp = h.empty_field(lat, fp, nrhs), h.empty_field(lat, fp, nrhs)
    dots = torch.full((nrhs,), float("nan"), dtype=torch.float64, device="cuda")
    ws = h.empty_workspace(h.hisq_apply_m_dot_workspace_bytes(lat, nrhs))
    h.hisq_apply_m_dot(lat, lp, fp, mass, links, inp, out, tmp, dots, ws, nrhs, ctx=ctx)
    got = h.unpack_field_to_host(lat, fp, out, nrhs)
    ref, dref = _m_dot_reference(w, lp, fp, mass, w["src"])
    _check_m_dot(got, dots.cpu().numpy(), ref, dref, lp, (lp, fp, variant))


def test_apply_m_dot_fp16n_links_fp32_fields_every_shape(gpu_lib, fields):
    """The FP16N-link, FP32-field operator of FP16N CG (D_oe plain, D_eo with
    the fused dot) in every launch shape the autotuner may pick."""
    h = gpu_lib
    dims, t_bc, nrhs, mass = (6, 4, 8, 10), -1, 3, 0.05
    w = fields(dims, t_bc, nrhs, "smooth")
    lat = h.lattice(dims, t_bc)
    ctx = h.Context(0)
    links = h.pack_links_from_host(lat, "fp16n", w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, "fp32", w["src"])
    ref, dref = _m_dot_reference(w, "fp16n", "fp32", mass, w["src"])
    ws = h.empty_workspace(h.hisq_apply_m_dot_workspace_bytes(lat, nrhs))
    for shape in _all_shapes(nrhs):
        h.hisq_set_dslash_shape(lat, "fp16n", nrhs, shape, ctx)
        out, tmp = h.empty_field(lat, "fp32", nrhs), h.empty_field(lat, "fp32", nrhs)
        out.fill_(0xFF)
        dots = torch.full((nrhs,), float("nan"), dtype=torch.float64, device="cuda")
        h.hisq_apply_m_dot(lat, "fp16n", "fp32", mass, links, inp, out, tmp, dots, ws, nrhs, ctx=ctx)
        got = h.unpack_field_to_host(lat, "fp32", out, nrhs)
        _check_m_dot(got, dots.cpu().numpy(), ref, dref, "fp16n", shape)


def test_apply_m_dot_rejects_bad_arguments(gpu_lib, fields):
    h = gpu_lib
    dims, t_bc = (4, 4, 4, 4), -1
    w = fields(dims, t_bc)
    lat = h.lattice(dims, t_bc)
    links = h.pack_links_from_host(lat, "fp32", w["fat"], w["naik"])
    a, b, c = (h.empty_field(lat, "fp64") for _ in range(3))
    dots = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = h.empty_workspace(h.hisq_apply_m_dot_workspace_bytes(lat, 1))
    with pytest.raises(h.HisqError) as e:        # FP32 links with FP64 fields: no such operator
        h.hisq_apply_m_dot(lat, "fp32", "fp64", 0.1, links, a, b, c, dots, ws)
    assert e.value.status == h.INVALID_ARG
    with pytest.raises(h.HisqError) as e:        # workspace too small
        h.hisq_apply_m_dot(lat, "fp32", "fp32", 0.1, links, a, b, c, dots, h.empty_workspace(8))
    assert e.value.status == h.WORKSPACE


def test_dslash_32x32x32x8_full_and_deterministic(gpu_lib):
    """Headline lattice, launch shape of the benchmark: full comparison with the
    oracle, and two applications bitwise identical."""
    h = gpu_lib
    w = gen.workload_2()
    dims, t_bc = w["dims"], w["t_bc"]
    lat = h.lattice(dims, t_bc)
    links = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
    src_o = gen.gaussian_half_field(gen.rng_for(2, 30), dims)[0]
    inp = h.pack_field_from_host(lat, "fp64", src_o)
    out1, out2 = h.empty_field(lat, "fp64"), h.empty_field(lat, "fp64")
    h.hisq_dslash(lat, "fp64", 0, links, inp, out1)
    h.hisq_dslash(lat, "fp64", 0, links, inp, out2)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)
    got = h.unpack_field_to_host(lat, "fp64", out1)[0]
    ref = O.lattice_from(w).D_eo(src_o)
    assert relerr(got, ref) <= 1e-13
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_dslash_rejects_bad_sizes(gpu_lib):
    h = gpu_lib
    lat = h.lattice((4, 4, 4, 4), 1)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        h.hisq_dslash(lat, "fp64", 0, small, small, small)


def _all_shapes(nrhs):
    out = []
    for var in (0, 1, 3):
        for nin in (1, 2, 4, 8):
            if nin > 1 and nin > nrhs:
                continue
            if var == 3 and nin > 2:
                continue
            for block in (64, 128, 256):
                for remap in (0, 1, 2):
                    out.append((var, nin, block, remap))
    return out


def fp16n_bound_ok(got, ref):
    """Element-wise bound of an FP16N output: each component within half a
    binary16 ulp of its site norm (the output's own rounding, 2^-12 n) plus
    the FP32 accumulation error.  Returns (ok, message)."""
    n = np.maximum(np.abs(ref.real), np.abs(ref.imag)).max(-1, keepdims=True)
    bound = (2.0 ** -12 + 2e-6) * n + 1e-6 * np.abs(ref).max()
    err = np.maximum(np.abs(got.real - ref.real), np.abs(got.imag - ref.imag))
    if np.all(err <= bound):
        return True, ""
    worst = np.unravel_index(np.argmax(err / bound), err.shape)
    return False, (f"index {worst}: err {err[worst]:.3e} bound {bound[worst[:-1] + (0,)]:.3e}, "
                   f"components over: {int((err > bound).sum())}")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16n", "fp64r12", "fp32r12"])
def test_every_launch_shape_matches_oracle(gpu_lib, fields, prec):
    """All shapes the autotuner may pick, on a lattice whose site count is not
    a multiple of the block (ragged tail) and nrhs = 3 (partial N_inner).
    FP16N is held to the element-wise bound of its output format."""
    h = gpu_lib
    dims, t_bc, nrhs = (6, 4, 8, 10), -1, 3
    w = fields(dims, t_bc, nrhs)
    lat = h.lattice(dims, t_bc)
    ctx = h.Context(0)
    links = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, prec, w["src_o"])
    lat_q = O.quantized_lattice(O.lattice_from(w), prec)
    ref = lat_q.D_eo(O.quantize_field(w["src_o"], prec))
    for shape in _all_shapes(nrhs):
        h.hisq_set_dslash_shape(lat, prec, nrhs, shape, ctx)
        assert h.hisq_get_dslash_shape(lat, prec, nrhs, ctx) == shape
        out = h.empty_field(lat, prec, nrhs)
        out.fill_(0xFF)
        h.hisq_dslash(lat, prec, 0, links, inp, out, nrhs, ctx=ctx)
        got = h.unpack_field_to_host(lat, prec, out, nrhs)
        if prec == "fp16n":
            ok, msg = fp16n_bound_ok(got, ref)
            assert ok, (shape, msg)
        else:
            assert relerr(got, ref) <= (1e-13 if prec.startswith("fp64") else 1e-6), shape


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16n"])
@pytest.mark.parametrize("dims", [(6, 16, 8, 6), (4, 24, 16, 4)])
def test_zslab_bands_match_oracle(gpu_lib, fields, prec, dims):
    """Block order 2 with several right-hand sides sweeps each z-slab in bands
    of 8 y-rows (N_y = 16: two bands, N_y = 24: three; N_z = 16: two planes per
    slab).  Every shape in that order must give the oracle's result, and the
    same bits as the contiguous order of the same variant, NIN and block: the
    traversal only permutes sites."""
    h = gpu_lib
    t_bc, nrhs = -1, 5
    w = fields(dims, t_bc, nrhs)
    lat = h.lattice(dims, t_bc)
    ctx = h.Context(0)
    links = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, prec, w["src_o"])
    lat_q = O.quantized_lattice(O.lattice_from(w), prec)
    ref = lat_q.D_eo(O.quantize_field(w["src_o"], prec))
    tol = {"fp64": 1e-13, "fp32": 1e-6, "fp16n": 2e-3}[prec]
    for var in (0, 1):
        for nin in (1, 2, 4):
            for block in (64, 256):
                base = None
                for remap in (1, 2):
                    shape = (var, nin, block, remap)
                    h.hisq_set_dslash_shape(lat, prec, nrhs, shape, ctx)
                    out = h.empty_field(lat, prec, nrhs)
                    out.fill_(0xFF)
                    h.hisq_dslash(lat, prec, 0, links, inp, out, nrhs, ctx=ctx)
                    got = h.unpack_field_to_host(lat, prec, out, nrhs)
                    assert relerr(got, ref) <= tol, shape
                    if base is None:
                        base = out.clone()
                    else:
                        assert torch.equal(out, base), shape


def test_zslab_block_order_needs_nz_divisible_by_8(gpu_lib):
    h = gpu_lib
    ctx = h.Context(0)
    with pytest.raises(h.HisqError):
        h.hisq_set_dslash_shape(h.lattice((8, 8, 12, 8), -1), "fp64", 1, (0, 1, 128, 2), ctx)
    h.hisq_set_dslash_shape(h.lattice((8, 8, 16, 8), -1), "fp64", 1, (0, 1, 128, 2), ctx)


def test_autotuner_picks_a_supported_shape(gpu_lib, fields):
    h = gpu_lib
    dims, t_bc = (8, 8, 8, 8), -1
    w = fields(dims, t_bc)
    lat = h.lattice(dims, t_bc)
    ctx = h.Context(0)
    links = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, "fp64", w["src_o"][0])
    out = h.empty_field(lat, "fp64")
    h.hisq_tune_dslash(lat, "fp64", 1, links, inp, out, ctx)
    shape = h.hisq_get_dslash_shape(lat, "fp64", 1, ctx)
    assert shape in _all_shapes(1) or shape[0] == 2, shape
    h.hisq_dslash(lat, "fp64", 0, links, inp, out, ctx=ctx)
    got = h.unpack_field_to_host(lat, "fp64", out)[0]
    assert relerr(got, O.lattice_from(w).D_eo(w["src_o"][0])) <= 1e-13


def test_stream_read_xors_every_word(gpu_lib):
    """The read-only bandwidth reference touches every 32-bit word: block b's
    sink word is the XOR of its 16 KiB (ragged last block included)."""
    h = gpu_lib
    n = 16 * (3 * 1024 + 517)
    src = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
    words = h.hisq_stream_read_sink_words(n)
    assert words == 4
    sink = torch.zeros(words + 4, dtype=torch.int32, device="cuda")
    h.hisq_stream_read(src, sink, n)
    torch.cuda.synchronize()
    w32 = src.cpu().numpy().view(np.uint32)
    want = [np.bitwise_xor.reduce(w32[b * 4096:(b + 1) * 4096]) for b in range(words)]
    got = sink.cpu().numpy().view(np.uint32)
    assert list(got[:words]) == want
    assert int(sink[words:].count_nonzero()) == 0


def test_stream_copy_is_exact(gpu_lib):
    """The bandwidth-reference copy moves every byte, including a ragged tail
    shorter than one block's 16 KiB."""
    h = gpu_lib
    n = 16 * (3 * 1024 + 517)
    src = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros(n + 64, dtype=torch.uint8, device="cuda")
    h.hisq_stream_copy(src, dst, n)
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src)
    assert int(dst[n:].count_nonzero()) == 0


# ---------------------------------------------------------------------------
# LDS-staged neighbours (variant 2): blocks of 8 y-rows x N_x/2 sites, x- and
# y-hop neighbour vectors read from LDS.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32r12", "fp64w14"])
@pytest.mark.parametrize("dims,t_bc,nrhs", [((16, 8, 8, 4), -1, 3), ((32, 16, 8, 6), 1, 5)])
@pytest.mark.parametrize("nin", [1, 2, 4])
def test_lds_staged_dslash_matches_oracle(gpu_lib, fields, prec, dims, t_bc, nrhs, nin):
    """Both parities, every column against the oracle on the stored formats;
    ragged groups of right-hand sides (nrhs not a multiple of nin)."""
    h = gpu_lib
    w = fields(dims, t_bc, nrhs)
    lat = h.lattice(dims, t_bc)
    ctx = h.Context(0)
    h.hisq_set_dslash_shape(lat, prec, nrhs, (2, nin, 64, 0), ctx)
    got_shape = h.hisq_get_dslash_shape(lat, prec, nrhs, ctx)
    assert got_shape[0] == 2 and got_shape[2] == 4 * dims[0] and got_shape[3] == 2
    links = h.pack_links_from_host(lat, prec, w["fat"], w["naik"])
    q = O.quantized_lattice(O.lattice_from(w), prec)
    for parity in (0, 1):
        src = w["src_o"] if parity == 0 else w["src"]
        inp = h.pack_field_from_host(lat, prec, src)
        out = h.empty_field(lat, prec, nrhs)
        out.fill_(0xFF)
        h.hisq_dslash(lat, prec, parity, links, inp, out, nrhs, ctx=ctx)
        got = h.unpack_field_to_host(lat, prec, out, nrhs)
        srcq = O.quantize_field(src, prec)
        ref = np.stack([q.D_eo(s) if parity == 0 else q.D_oe(s) for s in srcq])
        tol = 1e-13 if prec.startswith("fp64") else 2e-6
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (parity, np.abs(got - ref).max())


@pytest.mark.parametrize("lp,fp", [("fp64", "fp64"), ("fp32", "fp32"), ("fp16n", "fp32")])
def test_lds_staged_apply_m_dot(gpu_lib, fields, lp, fp):
    """The epilogues (m^2 y - D x and the fused dot) of the staged variant, and
    the FP16N-link x FP32-field pair of FP16N CG."""
    h = gpu_lib
    dims, t_bc, nrhs, mass = (16, 8, 8, 4), -1, 3, 0.1
    w = fields(dims, t_bc, nrhs, "smooth")
    lat = h.lattice(dims, t_bc)
    ctx = h.Context(0)
    h.hisq_set_dslash_shape(lat, lp, nrhs, (2, 2, 64, 2), ctx)
    links = h.pack_links_from_host(lat, lp, w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, fp, w["src"])
    out, tmp = h.empty_field(lat, fp, nrhs), h.empty_field(lat, fp, nrhs)
    dots = torch.full((nrhs,), float("nan"), dtype=torch.float64, device="cuda")
    ws = h.empty_workspace(h.hisq_apply_m_dot_workspace_bytes(lat, nrhs))
    h.hisq_apply_m_dot(lat, lp, fp, mass, links, inp, out, tmp, dots, ws, nrhs, ctx=ctx)
    got = h.unpack_field_to_host(lat, fp, out, nrhs)
    ref, dref = _m_dot_reference(w, lp, fp, mass, w["src"])
    _check_m_dot(got, dots.cpu().numpy(), ref, dref, lp, ("lds", lp, fp))


def test_lds_staged_shape_is_refused_where_it_does_not_fit(gpu_lib):
    h = gpu_lib
    ctx = h.Context(0)
    for dims in ((6, 8, 8, 4), (16, 6, 8, 4), (16, 8, 6, 4), (20, 8, 8, 4)):
        with pytest.raises(h.HisqError):
            h.hisq_set_dslash_shape(h.lattice(dims, -1), "fp32", 4, (2, 4, 64, 2), ctx)
    with pytest.raises(h.HisqError):   # FP64, 8 rhs per block at N_x = 64: 172 KiB of staging
        h.hisq_set_dslash_shape(h.lattice((64, 8, 8, 4), -1), "fp64", 8, (2, 8, 64, 2), ctx)
