"""GPU PTC preconditioner kernels against the FP64 oracle (oracle/ptc.py).

The GPU runs the network in FP32 (FP32 links, weights and activations, FP64
weight-gradient sums).  The oracle evaluates the same network in FP64 on the
FP32-rounded links, weights and inputs, so the difference is the FP32
arithmetic of three layers: relative 1e-5 is the bound used.
"""
import numpy as np
import pytest
import torch

import hisq_inputs as gen
from oracle import hisq as O
from oracle import ptc

pytestmark = pytest.mark.gpu

DIMS = (4, 6, 4, 8)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def f32(a):
    return O.quantize_fp32(a)


@pytest.fixture(scope="module")
def setup(gpu_lib):
    h = gpu_lib
    w = gen.workload_smooth(DIMS, 80, -1, 0.3, 4)
    lat = h.lattice(DIMS, -1)
    l32 = h.pack_links_from_host(lat, "fp32", w["fat"], w["naik"])
    X32 = f32(w["fat"])
    ws = h.empty_workspace(h.hisq_ptc_workspace_bytes(lat))
    weights = [np.asarray(f32(x)) for x in ptc.init_weights(np.random.default_rng(4), scale=0.6)]
    master, w32 = h.weights_to_device(weights)
    return h, w, lat, l32, X32, ws, weights, master, w32


def test_forward_matches_oracle(setup):
    h, w, lat, l32, X32, ws, weights, master, w32 = setup
    r = f32(w["src"][0])
    inp = h.pack_field_from_host(lat, "fp32", r)
    out = h.empty_field(lat, "fp32")
    h.hisq_ptc_forward(lat, l32, w32, inp, out, ws)
    got = h.unpack_field_to_host(lat, "fp32", out)[0]
    ref, _ = ptc.network_forward(DIMS, -1, X32, weights, r)
    assert rel(got, ref) <= 1e-5


def test_identity_weights_give_identity(setup):
    h, w, lat, l32, X32, ws, *_ = setup
    master, w32 = h.weights_to_device(ptc.identity_weights())
    r = f32(w["src"][1])
    inp = h.pack_field_from_host(lat, "fp32", r)
    out = h.empty_field(lat, "fp32")
    h.hisq_ptc_forward(lat, l32, w32, inp, out, ws)
    np.testing.assert_array_equal(h.unpack_field_to_host(lat, "fp32", out)[0], r)


def test_backward_matches_oracle(setup):
    h, w, lat, l32, X32, ws, weights, master, w32 = setup
    r = f32(w["src"][2])
    gout = f32(gen.gaussian_half_field(gen.rng_for(80, 30), DIMS)[0])
    inp = h.pack_field_from_host(lat, "fp32", r)
    out = h.empty_field(lat, "fp32")
    h.hisq_ptc_forward(lat, l32, w32, inp, out, ws)
    g_dev = h.pack_field_from_host(lat, "fp32", gout)
    gin = h.empty_field(lat, "fp32")
    grad = torch.zeros(2 * h.HISQ_PTC_NWEIGHTS, dtype=torch.float64, device="cuda")
    h.hisq_ptc_backward(lat, l32, w32, g_dev, gin, grad, ws)
    _, acts = ptc.network_forward(DIMS, -1, X32, weights, r)
    gws, gin_ref = ptc.network_backward(DIMS, -1, X32, weights, acts, gout)
    got_w = h.weights_from_device(grad)
    for a, b in zip(got_w, gws):
        assert rel(a, b) <= 1e-5
    assert rel(h.unpack_field_to_host(lat, "fp32", gin)[0], gin_ref) <= 1e-5
    # gradients accumulate: a second call doubles them
    h.hisq_ptc_backward(lat, l32, w32, g_dev, gin, grad, ws)
    for a, b in zip(h.weights_from_device(grad), gws):
        assert rel(a, 2 * b) <= 1e-5


def test_gauge_covariance_on_gpu(setup):
    h, w, lat, l32, X32, ws, weights, master, w32 = setup
    g = gen.gauge_transform(DIMS, gen.rng_for(80, gen.FIELD_GAUGE))
    Xg = np.empty_like(w["fat"])
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        Xg[mu] = g @ w["fat"][mu] @ np.roll(g, -1, axis=ax).conj().swapaxes(-1, -2)
    lg = h.pack_links_from_host(lat, "fp32", Xg, w["naik"])
    ge = g[ptc.even_mask(DIMS)]
    r = w["src"][3]
    out1, out2 = h.empty_field(lat, "fp32"), h.empty_field(lat, "fp32")
    h.hisq_ptc_forward(lat, l32, w32, h.pack_field_from_host(lat, "fp32", r), out1, ws)
    h.hisq_ptc_forward(lat, lg, w32, h.pack_field_from_host(lat, "fp32", np.einsum("sab,sb->sa", ge, r)),
                       out2, ws)
    y = h.unpack_field_to_host(lat, "fp32", out1)[0]
    yg = h.unpack_field_to_host(lat, "fp32", out2)[0]
    assert rel(yg, np.einsum("sab,sb->sa", ge, y)) <= 1e-5


def test_train_step_matches_oracle(setup):
    h, w, lat, l32, X32, ws, weights, master, w32 = setup
    srcs = f32(w["src"][:2])
    sols = gen.gaussian_half_field(gen.rng_for(80, 40), DIMS, 2)
    master, w32 = h.weights_to_device(weights)
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    s32 = h.pack_field_from_host(lat, "fp32", srcs)
    s64 = h.pack_field_from_host(lat, "fp64", sols)
    mass = 0.2
    loss = h.hisq_ptc_train_step(lat, mass, l32, master, w32, m, v, 1, 2, s32, s64, ws, lr=1e-2)
    lat_q = O.quantized_lattice(O.lattice_from(w), "fp32")
    L_ref, g_ref = ptc.loss_and_grad(DIMS, -1, X32, weights, srcs, O.quantize_fp32(sols),
                                     lambda v: lat_q.M_e(mass, v))
    assert abs(loss - L_ref) <= 1e-5 * L_ref
    zeros = [np.zeros_like(x) for x in weights]
    w_ref, _, _ = ptc.adam_step(weights, g_ref, zeros, zeros, 1, lr=1e-2)
    for a, b in zip(h.weights_from_device(master), w_ref):
        # first Adam step moves each part by ~lr sign(g): compare the update
        assert np.abs(a - b).max() <= 1e-6 + 1e-4 * 1e-2


def test_adam_kernel_three_steps_carry_moments(setup):
    """hisq_ptc_adam_step over three steps with changing gradients: weights,
    both moments (re and im parts as separate parameters) and the FP32 copy
    equal the oracle's FP64 Adam to rounding."""
    h, w, lat, l32, X32, ws, weights, master, w32 = setup
    rng = np.random.default_rng(11)
    wts = [x.astype(np.complex128) for x in weights]
    dev_w, dev_w32 = h.weights_to_device(wts)
    dev_m, dev_v = torch.zeros_like(dev_w), torch.zeros_like(dev_w)
    m_ref = [np.zeros_like(x) for x in wts]
    v_ref = [np.zeros_like(x) for x in wts]
    for step in (1, 2, 3):
        g = [rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape) for x in wts]
        g_dev, _ = h.weights_to_device(g)
        h.hisq_ptc_adam_step(dev_w, dev_w32, g_dev, dev_m, dev_v, step, lr=1e-2, beta1=0.8, beta2=0.95)
        wts, m_ref, v_ref = ptc.adam_step(wts, g, m_ref, v_ref, step, lr=1e-2, beta1=0.8, beta2=0.95)
        torch.cuda.synchronize()
        for got, ref in ((dev_w, wts), (dev_m, m_ref), (dev_v, v_ref)):
            for a, b in zip(h.weights_from_device(got), ref):
                np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)
        np.testing.assert_array_equal(dev_w32.cpu().numpy(), dev_w.to(torch.float32).cpu().numpy())


def test_train_step_three_steps_matches_oracle(setup):
    """Three training steps on one batch.  Before each step the weights and
    Adam moments are read from the GPU; the oracle computes the loss and the
    FP64 gradient at those weights (FP32-rounded, as the kernels use them) and
    one Adam step from those moments.  The GPU's loss, new weights and new
    moments must agree: the carried moments of steps 2 and 3 are pinned, not
    only the sign-like first step."""
    h, w, lat, l32, X32, ws, weights, master, w32 = setup
    srcs = f32(w["src"][:2])
    sols = gen.gaussian_half_field(gen.rng_for(80, 40), DIMS, 2)
    master, w32 = h.weights_to_device(weights)
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    s32 = h.pack_field_from_host(lat, "fp32", srcs)
    s64 = h.pack_field_from_host(lat, "fp64", sols)
    mass, lr = 0.2, 1e-2
    lat_q = O.quantized_lattice(O.lattice_from(w), "fp32")
    A = lambda v_: lat_q.M_e(mass, v_)  # noqa: E731
    for step in (1, 2, 3):
        w_prev = h.weights_from_device(master)
        m_prev = h.weights_from_device(m)
        v_prev = h.weights_from_device(v)
        loss = h.hisq_ptc_train_step(lat, mass, l32, master, w32, m, v, step, 2, s32, s64, ws, lr=lr)
        L_ref, g_ref = ptc.loss_and_grad(DIMS, -1, X32, [f32(x) for x in w_prev], srcs, O.quantize_fp32(sols), A)
        assert abs(loss - L_ref) <= 1e-5 * L_ref, (step, loss, L_ref)
        w_ref, m_ref, v_ref = ptc.adam_step(w_prev, g_ref, m_prev, v_prev, step, lr=lr)
        for a, b in zip(h.weights_from_device(m), m_ref):
            assert rel(a, b) <= 1e-5, step
        for a, b in zip(h.weights_from_device(v), v_ref):
            assert rel(a, b) <= 1e-5, step
        for a, b, p in zip(h.weights_from_device(master), w_ref, w_prev):
            # each update is ~lr per part; FP32 gradients move it by <= 1e-4 lr
            assert np.abs(a - b).max() <= 1e-6 + 1e-4 * lr, step
            assert np.abs(b - p).max() >= 0.5 * lr, step


def test_fcg_identity_preconditioner(gpu_lib):
    """With N = identity, flexible CG is CG: same tolerance, similar iterations."""
    h = gpu_lib
    w = gen.workload_smooth((8, 8, 4, 8), 81, -1, 0.3, 1)
    lat = h.lattice(w["dims"], -1)
    l64 = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
    l32 = h.pack_links_from_host(lat, "fp32", w["fat"], w["naik"])
    b = h.pack_field_from_host(lat, "fp64", w["src"][0])
    master, w32 = h.weights_to_device(ptc.identity_weights())
    x = h.empty_field(lat, "fp64")
    x.zero_()
    ws = h.empty_workspace(h.hisq_fcg_workspace_bytes(lat))
    st, info = h.hisq_fcg(lat, 0.05, l64, l32, w32, b, x, 1e-10, 20000, ws)
    assert st == h.OK, info
    xs = h.unpack_field_to_host(lat, "fp64", x)[0]
    assert O.true_residual(O.lattice_from(w), 0.05, w["src"][0], xs) <= 1e-10
    x2 = h.empty_field(lat, "fp64")
    x2.zero_()
    wsc = h.empty_workspace(h.hisq_cg_workspace_bytes(lat, "fp32", 1, 0))
    st2, info2 = h.hisq_cg(lat, 0.05, l64, l32, "fp32", 1, b, x2, 1e-10, 20000, wsc)
    assert st2 == h.OK
    assert abs(info["iterations"] - info2[0]["iterations"]) <= 0.15 * info2[0]["iterations"] + 5


def test_trained_network_in_flexible_cg(gpu_lib):
    """Train on (source, solution) pairs from the plain solver (the loss must
    fall), then solve held-out sources with FCG + PTC to the FP64 true residual
    and report its iterations against plain reliable-update CG.  The gain is
    measured, not asserted: on this light-mass operator a local linear network
    does not beat CG (see the iteration counts printed)."""
    h = gpu_lib
    dims, m = (8, 8, 8, 16), 0.05
    w = gen.workload_smooth(dims, 82, -1, 0.3, 0)
    lat = h.lattice(dims, -1)
    l64 = h.pack_links_from_host(lat, "fp64", w["fat"], w["naik"])
    l32 = h.pack_links_from_host(lat, "fp32", w["fat"], w["naik"])
    ntrain, ntest = 64, 4
    srcs = gen.gaussian_half_field(gen.rng_for(82, 3), dims, ntrain)
    test_srcs = gen.gaussian_half_field(gen.rng_for(82, 4), dims, ntest)
    wsc = h.empty_workspace(h.hisq_cg_workspace_bytes(lat, "fp32", 16, 0))
    sols = []
    for k in range(0, ntrain, 16):
        b = h.pack_field_from_host(lat, "fp64", srcs[k:k + 16])
        x = h.empty_field(lat, "fp64", 16)
        x.zero_()
        st, _ = h.hisq_cg(lat, m, l64, l32, "fp32", 16, b, x, 1e-8, 20000, wsc)
        assert st == h.OK
        sols.append(x)
    sol64 = torch.cat(sols)
    src32 = torch.cat([h.pack_field_from_host(lat, "fp32", srcs[k:k + 16]) for k in range(0, ntrain, 16)])
    master, w32 = h.weights_to_device(ptc.init_weights(np.random.default_rng(0), scale=0.05))
    mom, var = torch.zeros_like(master), torch.zeros_like(master)
    ws = h.empty_workspace(h.hisq_ptc_workspace_bytes(lat))
    fb32, fb64 = h.hisq_field_bytes(lat, "fp32", 1), h.hisq_field_bytes(lat, "fp64", 1)
    losses = []
    step = 0
    for epoch in range(40):
        for k in range(0, ntrain, 16):
            step += 1
            losses.append(h.hisq_ptc_train_step(lat, m, l32, master, w32, mom, var, step, 16,
                                                src32[k * fb32:(k + 16) * fb32],
                                                sol64[k * fb64:(k + 16) * fb64], ws, lr=3e-3))
    assert losses[-1] < 0.8 * losses[0], losses[::16]
    wsf = h.empty_workspace(h.hisq_fcg_workspace_bytes(lat))
    it_fcg, it_cg = [], []
    lat_o = O.lattice_from(w)
    for j in range(ntest):
        b = h.pack_field_from_host(lat, "fp64", test_srcs[j])
        x = h.empty_field(lat, "fp64")
        x.zero_()
        st, info = h.hisq_fcg(lat, m, l64, l32, w32, b, x, 1e-10, 20000, wsf)
        assert st == h.OK
        assert O.true_residual(lat_o, m, test_srcs[j], h.unpack_field_to_host(lat, "fp64", x)[0]) <= 1e-10
        it_fcg.append(info["iterations"])
        x.zero_()
        st, info2 = h.hisq_cg(lat, m, l64, l32, "fp32", 1, b, x, 1e-10, 20000, wsc)
        it_cg.append(info2[0]["iterations"])
    print(f"\nPTC loss {losses[0]:.3f} -> {losses[-1]:.3f}; held-out iterations FCG+PTC {it_fcg} vs CG {it_cg}; "
          f"ratio CG/FCG {np.mean(it_cg) / np.mean(it_fcg):.3f}")
