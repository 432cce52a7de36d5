"""FP64 oracle of the parallel-transport convolution (PTC) preconditioner.

TEST INFRASTRUCTURE ONLY (tests, the smoke check, the benchmark's CPU
baseline).  Shares no code with the GPU library.

The paper has no learned preconditioner; this follows the gauge-equivariant
parallel-transport convolution of Lehner and Wettig (arXiv:2302.05419), with
the fat links X as the connection, inside flexible CG (Notay, SIAM J. Sci.
Comput. 22 (2000) 1444).

Layer:   out_c(x) = sum_{c'} sum_{p in P} w[c, c', p] (T_p in_{c'})(x)
Paths:   P = (0, +0, -0, +1, -1, +2, -2, +3, -3); path index 0 is the identity,
         1 + 2 mu is the hop +mu and 2 + 2 mu the hop -mu.
         (T_{+mu} psi)(x) = X_mu(x) psi(x+mu)
         (T_{-mu} psi)(x) = X_mu(x-mu)^+ psi(x-mu)
         each with the spinor boundary sign on a hop that wraps in time.
Network: channels 1 -> 8 -> 8 -> 1, no bias, no nonlinearity.  The input is
         the even-site residual extended by zero to the odd sites; the output
         is read back on the even sites.

Fields here are whole-lattice arrays of shape (C, Nt, Nz, Ny, Nx, 3).
Gradients of a real loss L with respect to a complex z are returned as
dL/dRe z + i dL/dIm z.
"""
from __future__ import annotations

import numpy as np

NPATH = 9
CHANNELS = (1, 8, 8, 1)
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}   # axis of (Nt, Nz, Ny, Nx) moved along by mu


def _links(X, dims):
    nx, ny, nz, nt = dims
    return np.asarray(X).reshape(4, nt, nz, ny, nx, 3, 3)


def _edge(n, ax, idx):
    sl = [slice(None)] * 4
    sl[ax] = idx
    return tuple(sl)


def transport(dims, t_bc, X, psi, path: int) -> np.ndarray:
    """T_p psi for one field psi of shape (Nt, Nz, Ny, Nx, 3)."""
    if path == 0:
        return psi.copy()
    mu = (path - 1) // 2
    forward = (path - 1) % 2 == 0
    ax = _AXIS[mu]
    n = psi.shape[ax]
    U = _links(X, dims)[mu]
    if forward:
        shifted = np.roll(psi, -1, axis=ax)          # psi(x + mu)
        if mu == 3:
            shifted[_edge(n, ax, n - 1)] *= t_bc     # hop from the last slice wraps
        return np.einsum("...ab,...b->...a", U, shifted)
    u = np.einsum("...ba,...b->...a", U.conj(), psi)  # X_mu(y)^+ psi(y)
    shifted = np.roll(u, 1, axis=ax)                  # evaluated at y = x - mu
    if mu == 3:
        shifted[_edge(n, ax, 0)] *= t_bc             # hop from the first slice wraps
    return shifted


def adjoint_path(path: int) -> int:
    """T_p^+ = T_{p'}: the hop +mu is adjoint to the hop -mu."""
    if path == 0:
        return 0
    return path + 1 if (path - 1) % 2 == 0 else path - 1


def layer_forward(dims, t_bc, X, w, inp):
    """w: (Cout, Cin, 9) complex; inp: (Cin, ...) -> (Cout, ...)."""
    cout, cin, _ = w.shape
    out = np.zeros((cout,) + inp.shape[1:], dtype=np.complex128)
    for ci in range(cin):
        for p in range(NPATH):
            tp = transport(dims, t_bc, X, inp[ci], p)
            for co in range(cout):
                out[co] += w[co, ci, p] * tp
    return out


def layer_backward(dims, t_bc, X, w, inp, g_out):
    """Gradients (g_in, g_w) of a real loss through one layer."""
    cout, cin, _ = w.shape
    g_in = np.zeros_like(inp)
    g_w = np.zeros_like(w)
    for ci in range(cin):
        for p in range(NPATH):
            tp = transport(dims, t_bc, X, inp[ci], p)
            for co in range(cout):
                g_w[co, ci, p] = np.vdot(tp.ravel(), g_out[co].ravel())
    for ci in range(cin):
        for p in range(NPATH):
            acc = np.zeros_like(inp[ci])
            for co in range(cout):
                acc += np.conj(w[co, ci, p]) * g_out[co]
            g_in[ci] += transport(dims, t_bc, X, acc, adjoint_path(p))
    return g_in, g_w


def even_mask(dims) -> np.ndarray:
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    return (x + y + z + t) % 2 == 0


def embed_even(dims, half) -> np.ndarray:
    """(V/2, 3) even-site field -> (1, Nt, Nz, Ny, Nx, 3) whole-lattice field."""
    nx, ny, nz, nt = dims
    full = np.zeros((nt, nz, ny, nx, 3), dtype=np.complex128)
    full[even_mask(dims)] = half
    return full[None]


def restrict_even(dims, full) -> np.ndarray:
    return np.ascontiguousarray(full[0][even_mask(dims)])


def init_weights(rng: np.random.Generator, scale: float = 0.1):
    """Identity-path-dominated initial weights for the 1->8->8->1 network."""
    ws = []
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        g = rng.standard_normal((cout, cin, NPATH, 2)) * scale / np.sqrt(cin * NPATH)
        w = g[..., 0] + 1j * g[..., 1]
        w[:, :, 0] += 1.0 / np.sqrt(cin * cout)
        ws.append(w)
    return ws


def identity_weights():
    """Weights with N = identity: only the identity path, one channel carried."""
    ws = []
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        w = np.zeros((cout, cin, NPATH), dtype=np.complex128)
        w[0, 0, 0] = 1.0
        ws.append(w)
    return ws


def network_forward(dims, t_bc, X, ws, r_even):
    """N(r) on even sites; also returns the layer inputs for the backward pass."""
    h = embed_even(dims, r_even)
    acts = [h]
    for w in ws:
        h = layer_forward(dims, t_bc, X, w, h)
        acts.append(h)
    return restrict_even(dims, h), acts


def network_backward(dims, t_bc, X, ws, acts, g_out_even):
    """Weight gradients (and input gradient, even sites) for dL/dRe + i dL/dIm."""
    g = embed_even(dims, g_out_even)
    gws = [None] * len(ws)
    for li in range(len(ws) - 1, -1, -1):
        g, gws[li] = layer_backward(dims, t_bc, X, ws[li], acts[li], g)
    return gws, restrict_even(dims, g)


def loss_and_grad(dims, t_bc, X, ws, srcs, sols, apply_A):
    """L = (1/B) sum_i <e_i, A e_i> / <x_i, b_i>,  e_i = N(b_i) - x_i.

    The error of the network's approximation to x_i = A^-1 b_i measured in the
    A (energy) norm that CG minimises, relative to the energy norm of x_i
    (<x, A x> = <x, b>).  apply_A is the even-site operator M_e.  Returns the
    loss and the weight gradients dL/dRe w + i dL/dIm w.
    """
    B = len(srcs)
    total = 0.0
    gsum = [np.zeros_like(w) for w in ws]
    for b, x in zip(srcs, sols):
        y, acts = network_forward(dims, t_bc, X, ws, b)
        e = y - x
        Ae = apply_A(e)
        c = np.vdot(x.ravel(), b.ravel()).real
        total += np.vdot(e.ravel(), Ae.ravel()).real / c
        gws, _ = network_backward(dims, t_bc, X, ws, acts, 2.0 * Ae / c / B)
        for k in range(len(ws)):
            gsum[k] += gws[k]
    return total / B, gsum


def adam_step(ws, gs, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update, real and imaginary parts treated as separate parameters.

    ``step`` counts from 1.  Returns new (ws, m, v); m and v are stored as
    complex arrays holding the real and imaginary moments side by side.
    """
    new_w, new_m, new_v = [], [], []
    for w, g, mk, vk in zip(ws, gs, m, v):
        gr = np.stack([g.real, g.imag])
        mr = np.stack([mk.real, mk.imag]) * beta1 + (1 - beta1) * gr
        vr = np.stack([vk.real, vk.imag]) * beta2 + (1 - beta2) * gr * gr
        mh = mr / (1 - beta1 ** step)
        vh = vr / (1 - beta2 ** step)
        upd = lr * mh / (np.sqrt(vh) + eps)
        new_w.append(w - (upd[0] + 1j * upd[1]))
        new_m.append(mr[0] + 1j * mr[1])
        new_v.append(vr[0] + 1j * vr[1])
    return new_w, new_m, new_v


def fcg(lat, mass, b, precond, tol, max_iter, x0=None):
    """Flexible CG with one-vector truncation (Notay 2000).

    p_{k+1} = z_{k+1} - (<q_k, z_{k+1}> / <q_k, p_k>) p_k,  q_k = A p_k, and the
    step alpha_k = <p_k, r_k> / <p_k, q_k> minimises the A-norm error along p_k.
    Stops on the FP64 true residual.  Returns (x, status, iterations, true_res).
    """
    from .hisq import norm, vdot, OK, NOT_CONVERGED, BREAKDOWN
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    A = lambda v: lat.M_e(mass, v)  # noqa: E731
    bn = norm(b)
    r = b - A(x)
    z = precond(r)
    p = z.copy()
    for k in range(1, max_iter + 1):
        q = A(p)
        pq = vdot(p, q)
        if not np.isfinite(pq.real) or pq.real <= 0.0:
            return x, BREAKDOWN, k, norm(b - A(x)) / bn
        alpha = vdot(p, r) / pq
        x = x + alpha * p
        r = r - alpha * q
        if norm(r) <= tol * bn:
            r = b - A(x)
            if norm(r) <= tol * bn:
                return x, OK, k, norm(r) / bn
        z = precond(r)
        beta = vdot(q, z) / pq
        p = z - beta * p
    return x, NOT_CONVERGED, max_iter, norm(b - A(x)) / bn
