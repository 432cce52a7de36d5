"""The allocation-free M_e entry point (block partials in the library's static
device scratch) against hisq_apply_m_dot with a caller workspace: the same
kernels and launch shape, so outputs and dot products must agree bitwise.
Two calls in a row, the second on a smaller input, so a stale scratch or a
size mix-up between calls would show; and an oversized call is refused on the
host."""
import numpy as np
import pytest
import torch

import hisq_inputs as gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fields():
    def get(dims, t_bc, nsrc, kind, seed):
        return gen.workload_smooth(dims, 400 + seed, t_bc, 0.3, nsrc)
    return get


def _run_pair(h, fields, dims, t_bc, lp, fp, nrhs, mass, seed):
    w = fields(dims, t_bc, nrhs, "smooth", seed)
    lat = h.lattice(dims, t_bc)
    links = h.pack_links_from_host(lat, lp, w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, fp, w["src"])
    # reference: the workspace entry point
    out_ref, tmp_ref = h.empty_field(lat, fp, nrhs), h.empty_field(lat, fp, nrhs)
    dots_ref = torch.full((nrhs,), float("nan"), dtype=torch.float64, device="cuda")
    ws = h.empty_workspace(h.hisq_apply_m_dot_workspace_bytes(lat, nrhs))
    h.hisq_apply_m_dot(lat, lp, fp, mass, links, inp, out_ref, tmp_ref, dots_ref, ws, nrhs)
    # allocation-free entry point
    out, tmp = h.empty_field(lat, fp, nrhs), h.empty_field(lat, fp, nrhs)
    out.fill_(0x5A)
    dots = torch.full((nrhs,), float("nan"), dtype=torch.float64, device="cuda")
    h.hisq_apply_m_dot_noalloc(lat, lp, fp, mass, links, inp, out, tmp, dots, nrhs)
    torch.cuda.synchronize()
    assert torch.equal(out, out_ref), (dims, lp, fp, nrhs)
    a, b = dots.cpu().numpy(), dots_ref.cpu().numpy()
    assert np.all(np.isfinite(a)), a
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (a, b)
    return a


@pytest.mark.parametrize("lp,fp", [("fp64", "fp64"), ("fp16n", "fp32")])
def test_noalloc_matches_workspace_entry_point(gpu_lib, fields, lp, fp):
    h = gpu_lib
    print(f"noalloc {lp}/{fp}: 8x8x8x8 nrhs 4, then 4x4x6x4 nrhs 1", flush=True)
    big = _run_pair(h, fields, (8, 8, 8, 8), -1, lp, fp, 4, 0.1, 1)
    small = _run_pair(h, fields, (4, 4, 6, 4), 1, lp, fp, 1, 0.2, 2)
    assert big.shape == (4,) and small.shape == (1,)


def test_noalloc_with_context_and_oversized_call(gpu_lib, fields):
    h = gpu_lib
    ctx = h.Context(0)
    dims, t_bc, nrhs = (6, 4, 8, 10), -1, 3
    w = fields(dims, t_bc, nrhs, "smooth", 3)
    lat = h.lattice(dims, t_bc)
    links = h.pack_links_from_host(lat, "fp32", w["fat"], w["naik"])
    inp = h.pack_field_from_host(lat, "fp32", w["src"])
    out_ref, tmp_ref = h.empty_field(lat, "fp32", nrhs), h.empty_field(lat, "fp32", nrhs)
    out, tmp = h.empty_field(lat, "fp32", nrhs), h.empty_field(lat, "fp32", nrhs)
    d_ref = torch.zeros(nrhs, dtype=torch.float64, device="cuda")
    d = torch.zeros(nrhs, dtype=torch.float64, device="cuda")
    ws = h.empty_workspace(h.hisq_apply_m_dot_workspace_bytes(lat, nrhs))
    h.hisq_set_dslash_shape(lat, "fp32", nrhs, (1, 2, 64, 1), ctx)  # four lanes per site, 16 sites per block
    h.hisq_apply_m_dot(lat, "fp32", "fp32", 0.05, links, inp, out_ref, tmp_ref, d_ref, ws, nrhs, ctx=ctx)
    h.hisq_apply_m_dot_noalloc(lat, "fp32", "fp32", 0.05, links, inp, out, tmp, d, nrhs, ctx=ctx)
    torch.cuda.synchronize()
    # three FP32 columns leave the second slot of the last column pair unused
    # (not written by the four-lanes-per-site kernel): compare the columns
    got = h.unpack_field_to_host(lat, "fp32", out, nrhs)
    ref = h.unpack_field_to_host(lat, "fp32", out_ref, nrhs)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    assert torch.equal(d, d_ref)
    # a call whose partials exceed the scratch is refused before any launch
    # (buffers of the right sizes all the same, so nothing could go out of
    # bounds even if the check were missing)
    big = h.lattice((32, 32, 32, 36), -1)
    nb = 16
    assert h.hisq_apply_m_dot_workspace_bytes(big, nb) > h.HISQ_NOALLOC_SCRATCH_BYTES
    ctx2 = h.Context(0)
    h.hisq_set_dslash_shape(big, "fp32", nb, (1, 2, 64, 1), ctx2)
    links_b = torch.zeros(h.hisq_links_bytes(big, "fp32"), dtype=torch.uint8, device="cuda")
    fb = [h.empty_field(big, "fp32", nb) for _ in range(3)]
    d_b = torch.zeros(nb, dtype=torch.float64, device="cuda")
    with pytest.raises(h.HisqError) as e:
        h.hisq_apply_m_dot_noalloc(big, "fp32", "fp32", 0.05, links_b, fb[0], fb[1], fb[2], d_b, nb, ctx=ctx2)
    assert e.value.status == h.WORKSPACE
