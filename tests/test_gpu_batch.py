"""GPU batched CG over independent lattices of different sizes, judged by the
FP64 oracle's true residual of every (or every sampled) problem."""
import numpy as np
import pytest
import torch

import hisq_inputs as gen
from oracle import hisq as O

pytestmark = pytest.mark.gpu


def build(h, ws_list, inner, tol=1e-10):
    items, keep = [], []
    for w in ws_list:
        lat = h.lattice(w["dims"], w["t_bc"])
        l64 = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
        lin = None if inner == "fp64" else h.pack_links_from_host(lat, inner, w["fat"], w["naik"])
        b = h.pack_field_from_host(lat, "fp64", w["src"][0])
        x = h.empty_field(lat, "fp64")
        x.zero_()
        items.append(dict(lat=lat, mass=w["mass"], links_f64=l64, links_inner=lin, b=b, x=x, tol=tol))
        keep += [l64, lin, b, x]
    probs = h.make_problems(items)
    ws = h.empty_workspace(h.hisq_cg_batch_workspace_bytes(probs, inner))
    return items, probs, ws, keep


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_batch_small_uneven(gpu_lib, inner):
    h = gpu_lib
    shapes = [(4, 4, 4, 4), (6, 4, 4, 8), (8, 8, 8, 8), (4, 4, 8, 6), (8, 8, 8, 8), (6, 6, 6, 4)]
    rng = np.random.default_rng(3)
    ws_list = []
    for k, d in enumerate(shapes):
        w = gen.workload_haar(d, 600 + k, -1 if k % 2 else +1)
        w["mass"] = float(rng.uniform(0.05, 0.2))
        ws_list.append(w)
    items, probs, ws, keep = build(h, ws_list, inner)
    st, info, lat_s = h.hisq_cg_batch(probs, inner, 20000, ws)
    assert st == h.OK, info
    for it, w, inf in zip(items, ws_list, info):
        x = h.unpack_field_to_host(it["lat"], "fp64", it["x"])[0]
        r = O.true_residual(O.lattice_from(w), w["mass"], w["src"][0], x)
        assert r <= 1e-10 and inf["true_residual"] <= 1e-10, (w["dims"], r, inf)
    assert all(l > 0 for l in lat_s)
    # the same problem solved alone by hisq_cg converges to the same tolerance
    it, w = items[2], ws_list[2]
    x1 = h.empty_field(it["lat"], "fp64")
    x1.zero_()
    ws1 = h.empty_workspace(h.hisq_cg_workspace_bytes(it["lat"], inner, 1, 0))
    st1, info1 = h.hisq_cg(it["lat"], w["mass"], it["links_f64"], it["links_inner"], inner, 1, it["b"], x1,
                           1e-10, 20000, ws1)
    assert st1 == h.OK
    assert abs(info1[0]["iterations"] - info[2]["iterations"]) <= 0.2 * info1[0]["iterations"] + 5


def test_batch_status_and_arguments(gpu_lib):
    h = gpu_lib
    ws_list = [dict(gen.workload_haar((4, 4, 4, 4), 700 + k, -1), mass=0.1) for k in range(2)]
    items, probs, ws, keep = build(h, ws_list, "fp64", tol=1e-12)
    st, info, _ = h.hisq_cg_batch(probs, "fp64", 3, ws)
    assert st == h.NOT_CONVERGED and all(i["iterations"] == 3 for i in info)
    small = h.empty_workspace(256)
    with pytest.raises(h.HisqError) as e:
        h.hisq_cg_batch(probs, "fp64", 10, small)
    assert e.value.status == h.WORKSPACE


def test_workload_uneven_batch_64(gpu_lib):
    """64 Haar-link solves on 8^4, 12^3x4, 16^3x8, 24^3x6 (24/20/12/8), masses
    U[0.01, 0.1], FP32 iterations with FP64 reliable updates, tol 1e-10."""
    h = gpu_lib
    ws_list = gen.workload_4()
    items, probs, ws, keep = build(h, ws_list, "fp32")
    torch.cuda.synchronize()
    st, info, lat_s = h.hisq_cg_batch(probs, "fp32", 40000, ws)
    assert st == h.OK, [i for i in info if i["true_residual"] > 1e-10]
    assert max(i["true_residual"] for i in info) <= 1e-10
    # oracle true residual of every one of the 64 solutions
    for k in range(len(items)):
        it, w = items[k], ws_list[k]
        x = h.unpack_field_to_host(it["lat"], "fp64", it["x"])[0]
        assert O.true_residual(O.lattice_from(w), w["mass"], w["src"][0], x) <= 1e-10, k
    # latencies end at each problem's confirmed solve, inside the batch's wall time
    assert all(0.0 < t <= info[0]["seconds"] for t in lat_s), lat_s
    lat_ms = np.array(lat_s) * 1e3
    print(f"\nbatch of 64: wall {info[0]['seconds']:.3f} s, latency p50 {np.percentile(lat_ms, 50):.1f} ms "
          f"p99 {np.percentile(lat_ms, 99):.1f} ms, iterations {min(i['iterations'] for i in info)}.."
          f"{max(i['iterations'] for i in info)}")


def test_batch_with_a_zero_source(gpu_lib):
    """A problem whose source is zero is done before the first iteration (x = 0)
    while the others iterate to their tolerance."""
    h = gpu_lib
    ws_list = [gen.workload_haar(d, 95 + k, -1) for k, d in enumerate([(4, 4, 4, 4), (4, 4, 6, 4), (6, 4, 4, 4)])]
    for w in ws_list:
        w["mass"] = 0.1
    ws_list[1]["src"] = np.zeros_like(ws_list[1]["src"])
    items, probs, ws, keep = build(h, ws_list, "fp32")
    st, info, lat_s = h.hisq_cg_batch(probs, "fp32", 20000, ws)
    assert st == h.OK, info
    assert info[1]["iterations"] == 0
    x1 = h.unpack_field_to_host(items[1]["lat"], "fp64", items[1]["x"])[0]
    assert np.all(x1 == 0)
    for j in (0, 2):
        w = ws_list[j]
        xj = h.unpack_field_to_host(items[j]["lat"], "fp64", items[j]["x"])[0]
        assert O.true_residual(O.lattice_from(w), 0.1, w["src"][0], xj) <= 1e-10


def test_batch_compaction_and_iteration_limit(gpu_lib):
    """Three easy problems finish early, so the work list is compacted to the
    remaining hard one, which then stops at the iteration limit: the easy ones
    meet the tolerance, and the hard one's reported true residual (formed on
    the restored full work list) is the oracle's for the x it returned."""
    h = gpu_lib
    dims = [(8, 8, 8, 8), (6, 4, 4, 4), (4, 4, 6, 4), (4, 6, 4, 4)]
    ws_list = [gen.workload_haar(d, 810 + k, -1) for k, d in enumerate(dims)]
    ws_list[0]["mass"] = 0.01
    for w in ws_list[1:]:
        w["mass"] = 3.0  # kappa ~ 8: a few dozen iterations
    items, probs, ws, keep = build(h, ws_list, "fp32")
    st, info, lat_s = h.hisq_cg_batch(probs, "fp32", 200, ws)
    assert st == h.NOT_CONVERGED
    assert info[0]["iterations"] == 200
    for k in range(4):
        it, w = items[k], ws_list[k]
        x = h.unpack_field_to_host(it["lat"], "fp64", it["x"])[0]
        r = O.true_residual(O.lattice_from(w), w["mass"], w["src"][0], x)
        if k == 0:
            assert r > 1e-10 and abs(r - info[0]["true_residual"]) <= 1e-9 * r, (r, info[0])
        else:
            assert r <= 1e-10 and info[k]["iterations"] < 100, (k, r, info[k])
