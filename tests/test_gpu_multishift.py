"""GPU multi-shift CG judged by the FP64 oracle: x_k = (M_e + sigma_k)^-1 b.

The oracle's definition solves each shift on its own; the GPU reaches the same
solutions from one Krylov space.  Every shift's true residual, recomputed by
the oracle, must meet its tolerance.
"""
import numpy as np
import pytest
import torch

import hisq_inputs as gen
from oracle import hisq as O

pytestmark = pytest.mark.gpu

SHIFTS14 = 10.0 ** (-5.0 + 5.0 * np.arange(14) / 13.0)


def run(h, w, inner, shifts, mass, tol=1e-10, max_iter=20000, src=None):
    dims, t_bc = w["dims"], w["t_bc"]
    lat = h.lattice(dims, t_bc)
    l64 = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
    lin = None if inner == "fp64" else h.pack_links_from_host(lat, inner, w["fat"], w["naik"])
    src = w["src"][0] if src is None else src
    b = h.pack_field_from_host(lat, "fp64", src)
    xs = [h.empty_field(lat, "fp64") for _ in shifts]
    ws = h.empty_workspace(h.hisq_cg_workspace_bytes(lat, inner, 1, len(shifts)))
    st, info = h.hisq_multishift_cg(lat, mass, l64, lin, inner, shifts, b, xs, tol, max_iter, ws)
    sols = [h.unpack_field_to_host(lat, "fp64", x)[0] for x in xs]
    return st, info, sols, (lat, l64, lin, b, xs, ws)


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_multishift_small(gpu_lib, inner):
    h = gpu_lib
    w = gen.workload_smooth((8, 4, 8, 8), 51, -1, 0.3, 1)
    m = 0.05
    shifts = [0.3, 0.0, 1e-3, 0.3, 2.0, 0.05]      # unsorted, with a duplicate
    st, info, sols, _ = run(h, w, inner, shifts, m)
    assert st == h.OK, info
    lat_o = O.lattice_from(w)
    for k, s in enumerate(shifts):
        r = O.true_residual(lat_o, m, w["src"][0], sols[k], shift=s)
        assert r <= 1e-10, (k, s, r)
        assert info[k]["true_residual"] <= 1e-10
    np.testing.assert_array_equal(sols[0], sols[3])     # duplicate shifts
    # the larger shifts converge earlier in the shared Krylov space
    assert info[4]["iterations"] <= info[1]["iterations"]


SHIFTS5 = [0.0, 1e-3, 0.05, 0.3, 2.0]
KRYLOV_CASES = [("haar", (8, 8, 8, 8), 61, 0.2), ("smooth", (8, 4, 8, 8), 51, 0.05)]


def _krylov_inputs(kind, dims, seed):
    if kind == "haar":
        return gen.workload_haar(dims, seed, -1)
    return gen.workload_smooth(dims, seed, -1, 0.3, 1)


@pytest.mark.parametrize("kind,dims,seed,m", KRYLOV_CASES)
def test_multishift_krylov_phase_fp64_needs_no_refinement(gpu_lib, kind, dims, seed, m):
    """The shared Krylov space alone (Jegerlehner's zeta, alpha_k, beta_k
    recurrences, FP64): every shifted iterate x_k at its freeze meets its
    tolerance by the oracle's FP64 true residual, and the full solver then
    refines no shift at all.  A wrong recurrence would leave the x_k far from
    (M_e + sigma_k)^-1 b and the refinement would have to do the work."""
    h = gpu_lib
    w = _krylov_inputs(kind, dims, seed)
    lat = h.lattice(w["dims"], w["t_bc"])
    l64 = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
    b = h.pack_field_from_host(lat, "fp64", w["src"][0])
    xs = [h.empty_field(lat, "fp64") for _ in SHIFTS5]
    ws = h.empty_workspace(h.hisq_cg_workspace_bytes(lat, "fp64", 1, len(SHIFTS5)))
    st, info = h.hisq_multishift_krylov(lat, m, l64, None, "fp64", SHIFTS5, b, xs, 1e-10, 20000, ws)
    assert st == h.OK, info
    lat_o = O.lattice_from(w)
    for k, s in enumerate(SHIFTS5):
        sol = h.unpack_field_to_host(lat, "fp64", xs[k])[0]
        r = O.true_residual(lat_o, m, w["src"][0], sol, shift=s)
        assert r <= 1e-10, (k, s, r)
        assert abs(info[k]["true_residual"] - r) <= 1e-3 * r
        assert info[k]["refine_iterations"] == 0
        assert info[k]["shared_iterations"] == info[k]["iterations"] > 0
    # larger shifts are better conditioned: frozen no later than smaller ones
    its = [i["shared_iterations"] for i in info]
    assert its == sorted(its, reverse=True), its
    st2, info2 = h.hisq_multishift_cg(lat, m, l64, None, "fp64", SHIFTS5, b, xs, 1e-10, 20000, ws)
    assert st2 == h.OK, info2
    for k in range(len(SHIFTS5)):
        assert info2[k]["refine_iterations"] == 0, (k, info2[k])
        assert info2[k]["shared_iterations"] == its[k]
        assert info2[k]["iterations"] == its[k]


@pytest.mark.parametrize("kind,dims,seed,m", KRYLOV_CASES)
def test_multishift_krylov_phase_fp32_matches_per_shift_solves(gpu_lib, kind, dims, seed, m):
    """With FP32 iteration vectors and links the Krylov iterates stall near
    FP32 precision, before any refinement: each x_k must still equal the
    oracle's independent per-shift solution to 1e-5 relative (an emulation of
    the same recurrences with FP32-rounded vectors lands at 1e-7 to 3e-7)."""
    h = gpu_lib
    w = _krylov_inputs(kind, dims, seed)
    lat = h.lattice(w["dims"], w["t_bc"])
    l64 = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
    l32 = h.pack_links_from_host(lat, "fp32", w["fat"], w["naik"])
    b = h.pack_field_from_host(lat, "fp64", w["src"][0])
    xs = [h.empty_field(lat, "fp64") for _ in SHIFTS5]
    ws = h.empty_workspace(h.hisq_cg_workspace_bytes(lat, "fp32", 1, len(SHIFTS5)))
    st, info = h.hisq_multishift_krylov(lat, m, l64, l32, "fp32", SHIFTS5, b, xs, 1e-10, 20000, ws)
    assert st in (h.OK, h.NOT_CONVERGED), info
    ref = O.multishift_reference(O.lattice_from(w), m, SHIFTS5, w["src"][0], 1e-12, 20000)
    for k in range(len(SHIFTS5)):
        assert ref[k].status == O.OK
        sol = h.unpack_field_to_host(lat, "fp64", xs[k])[0]
        err = np.linalg.norm(sol - ref[k].x) / np.linalg.norm(ref[k].x)
        assert err <= 1e-5, (k, err)
        assert info[k]["refine_iterations"] == 0 and info[k]["shared_iterations"] > 0


def test_multishift_single_shift_is_cg(gpu_lib):
    """nshift = 1 is plain CG: the shared Krylov phase (the two-reduction
    recurrence) needs no refinement and takes the iterations hisq_cg (the
    single-reduction recurrence, the same iterates in exact arithmetic) and
    the oracle's textbook CG take, to within rounding (+-2), and all three
    solutions agree."""
    h = gpu_lib
    w = gen.workload_haar((8, 8, 4, 8), 52, -1)
    st, info, sols, (lat, l64, lin, b, xs, ws) = run(h, w, "fp64", [0.0], 0.1)
    assert st == h.OK
    assert info[0]["refine_iterations"] == 0
    x = h.empty_field(lat, "fp64")
    x.zero_()
    ws2 = h.empty_workspace(h.hisq_cg_workspace_bytes(lat, "fp64", 1, 0))
    st2, info2 = h.hisq_cg(lat, 0.1, l64, None, "fp64", 1, b, x, 1e-10, 20000, ws2)
    assert st2 == h.OK
    ref = O.cg(O.lattice_from(w), 0.1, w["src"][0], 1e-10, 20000)
    assert abs(info2[0]["iterations"] - info[0]["iterations"]) <= 2, (info2[0], info[0])
    assert abs(info2[0]["iterations"] - ref.iterations) <= 2, (info2[0], ref.iterations)
    got = h.unpack_field_to_host(lat, "fp64", x)[0]
    lat_o = O.lattice_from(w)
    assert O.true_residual(lat_o, 0.1, w["src"][0], got) <= 1e-10
    assert O.true_residual(lat_o, 0.1, w["src"][0], sols[0]) <= 1e-10
    # condition number ~4e3 at m = 0.1: solutions within ~1e-6 of each other
    scale = np.linalg.norm(ref.x)
    assert np.linalg.norm(got - ref.x) <= 1e-5 * scale
    assert np.linalg.norm(sols[0] - ref.x) <= 1e-5 * scale


def test_multishift_per_shift_tolerances_and_errors(gpu_lib):
    h = gpu_lib
    w = gen.workload_smooth((4, 4, 8, 8), 53, -1, 0.3, 1)
    shifts = [0.0, 0.1, 1.0]
    tols = [1e-6, 1e-10, 1e-8]
    st, info, sols, (lat, l64, lin, b, xs, ws) = run(h, w, "fp64", shifts, 0.1, tol=tols)
    assert st == h.OK
    lat_o = O.lattice_from(w)
    for k, s in enumerate(shifts):
        assert O.true_residual(lat_o, 0.1, w["src"][0], sols[k], shift=s) <= tols[k]
    with pytest.raises(h.HisqError):   # m^2 + shift <= 0
        h.hisq_multishift_cg(lat, 0.1, l64, None, "fp64", [-0.02], b, xs[:1], 1e-8, 100, ws)
    with pytest.raises(h.HisqError):   # aliasing solutions
        h.hisq_multishift_cg(lat, 0.1, l64, None, "fp64", [0.0, 0.1], b, [xs[0], xs[0]], 1e-8, 100, ws)


def test_workload_48x48x48x12_multi_rhs_and_multishift(gpu_lib):
    """48^3x12 smooth links, m = 0.005: 16 right-hand sides in one batched
    FP32/FP64-reliable CG, and 14 log-spaced shifts in [1e-5, 1] to 1e-10.
    Oracle true residuals for all 16 right-hand sides and all 14 shifts."""
    h = gpu_lib
    w = gen.workload_3()
    dims, t_bc, m = w["dims"], w["t_bc"], w["mass"]
    lat = h.lattice(dims, t_bc)
    l64 = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
    l32 = h.pack_links_from_host(lat, "fp32", w["fat"], w["naik"])
    b = h.pack_field_from_host(lat, "fp64", w["src"])
    x = h.empty_field(lat, "fp64", 16)
    x.zero_()
    ws = h.empty_workspace(h.hisq_cg_workspace_bytes(lat, "fp32", 16, 0))
    st, info = h.hisq_cg(lat, m, l64, l32, "fp32", 16, b, x, 1e-10, 40000, ws)
    assert st == h.OK, info
    assert max(i["true_residual"] for i in info) <= 1e-10
    xs = h.unpack_field_to_host(lat, "fp64", x, 16)
    lat_o = O.lattice_from(w)
    for j in range(16):
        assert O.true_residual(lat_o, m, w["src"][j], xs[j]) <= 1e-10, j
    print(f"\n48^3x12 16-RHS: iterations {[i['iterations'] for i in info]}, {info[0]['seconds']:.3f} s")
    del x, ws
    b1 = h.pack_field_from_host(lat, "fp64", w["src"][0])
    xk = [h.empty_field(lat, "fp64") for _ in SHIFTS14]
    ws = h.empty_workspace(h.hisq_cg_workspace_bytes(lat, "fp32", 1, 14))
    st, info = h.hisq_multishift_cg(lat, m, l64, l32, "fp32", SHIFTS14, b1, xk, 1e-10, 40000, ws)
    assert st == h.OK, info
    for k, s in enumerate(SHIFTS14):
        sol = h.unpack_field_to_host(lat, "fp64", xk[k])[0]
        assert O.true_residual(lat_o, m, w["src"][0], sol, shift=s) <= 1e-10, k
    print(f"48^3x12 multishift: iterations {[i['iterations'] for i in info]}, {info[0]['seconds']:.3f} s")


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_multishift_32_shifts_refined_in_two_groups(gpu_lib, inner):
    """The maximum of 32 shifts: the refinement solves them as two 16-column
    multi-RHS groups, each column with its own shift and tolerance."""
    h = gpu_lib
    w = gen.workload_smooth((4, 4, 6, 8), 47, -1, 0.3, 1)
    shifts = list(10.0 ** (-4.0 + 4.0 * np.arange(32) / 31.0))
    tols = [1e-10 if k % 2 == 0 else 1e-8 for k in range(32)]
    st, info, sols, _ = run(h, w, inner, shifts, 0.05, tol=tols)
    assert st == h.OK, info
    lat_o = O.lattice_from(w)
    for k in range(32):
        assert O.true_residual(lat_o, 0.05, w["src"][0], sols[k], shift=shifts[k]) <= tols[k], k
        assert info[k]["iterations"] == info[k]["shared_iterations"] + info[k]["refine_iterations"]


def test_multishift_zero_source(gpu_lib):
    h = gpu_lib
    w = gen.workload_smooth((4, 4, 4, 4), 48, -1, 0.3, 1)
    st, info, sols, _ = run(h, w, "fp32", [0.0, 0.1, 1.0], 0.1, src=np.zeros_like(w["src"][0]))
    assert st == h.OK
    for s in sols:
        assert np.all(s == 0)
