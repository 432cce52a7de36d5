"""FP64 oracle: even/odd Dslash, the normal operator, CG and multi-shift CG.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline).  Shares no code with the GPU library.

Conventions follow the paper:

* lattice, links, colour vectors and boundary conditions: Sec. 3 "Physics
  modules" (links periodic, colour vectors periodic in space and, by default,
  antiperiodic in time);
* even/odd ordering: Sec. 4.3 "Indexing and fields" -- the sites of one parity
  in increasing lexicographic order (the paper's index floor(lex/2));
* the stencil: Sec. 5.1 "HISQ Dslash performance model" (evaluated by the C
  loop in ``hisq_oracle.c``);
* the solvers: Sec. 3.2 "Inverters" -- CG for A x = b with A Hermitian positive
  definite, and the multi-shift problem (A + sigma_k) x_k = b.

Here A is the even-site normal operator M_e = m^2 - D_eo D_oe.  D_eo maps odd
sites to even ones (the first index names the output parity) and D_oe the
reverse.  The multi-shift reference solves each shift on its own with plain CG:
the multi-shift method reaches the same solutions, so the oracle is their
definition.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _open(path: str):
    if not os.path.exists(path):
        raise RuntimeError(f"oracle library not built: {path}")
    lib_ = ctypes.CDLL(path)
    lib_.oracle_dslash.restype = ctypes.c_int
    lib_.oracle_dslash.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int]
    lib_.oracle_dslash_sites.restype = ctypes.c_int
    lib_.oracle_dslash_sites.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_long, ctypes.c_void_p]
    lib_.oracle_num_threads.restype = ctypes.c_int
    lib_.oracle_set_num_threads.restype = None
    lib_.oracle_set_num_threads.argtypes = [ctypes.c_int]
    return lib_


def lib():
    """The compiled C oracle (built by ``oracle/build.sh`` next to this file)."""
    global _lib
    if _lib is None:
        _lib = _open(LIB_PATH)
    return _lib


@contextlib.contextmanager
def substituted_library(path: str):
    """For the mutation check of the pins only: inside the block every oracle
    call goes to the C library at ``path`` (a build of a deliberately altered
    ``hisq_oracle.c``); the previous library is restored on exit."""
    global _lib
    saved = _lib
    _lib = _open(path)
    try:
        yield
    finally:
        _lib = saved


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of later oracle calls (timing only; results are the same)."""
    lib().oracle_set_num_threads(int(n))


# ---------------------------------------------------------------------------
# Lattice bookkeeping (Sec. 4.3)
# ---------------------------------------------------------------------------

def volume(dims) -> int:
    return int(np.prod(dims))


def site_parity(dims) -> np.ndarray:
    """Parity (x+y+z+t) mod 2 of every site, in lexicographic order."""
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    return ((x + y + z + t) % 2).ravel()


def parity_sites(dims, parity: int) -> np.ndarray:
    """Lexicographic indices of the sites of one parity, in increasing order."""
    return np.nonzero(site_parity(dims) == parity)[0]


def to_full(half: np.ndarray, dims, parity: int) -> np.ndarray:
    """(V/2, 3) field on one parity -> (V, 3) field, zero on the other parity."""
    full = np.zeros((volume(dims), 3), dtype=np.complex128)
    full[parity_sites(dims, parity)] = half
    return full


def from_full(full: np.ndarray, dims, parity: int) -> np.ndarray:
    return np.ascontiguousarray(full.reshape(volume(dims), 3)[parity_sites(dims, parity)])


def _links(U: np.ndarray, dims) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.complex128).reshape(4, volume(dims), 3, 3)
    return U


def _dims_arg(dims):
    return (ctypes.c_int * 4)(*[int(d) for d in dims])


# ---------------------------------------------------------------------------
# Dslash
# ---------------------------------------------------------------------------

def dslash_full(dims, t_bc: int, X, W, psi_full, out_parity: int = -1) -> np.ndarray:
    """D psi on the whole lattice; psi_full has shape (V, 3) (lexicographic)."""
    X = _links(X, dims)
    W = _links(W, dims)
    psi = np.ascontiguousarray(psi_full, dtype=np.complex128).reshape(volume(dims), 3)
    out = np.empty_like(psi)
    rc = lib().oracle_dslash(_dims_arg(dims), int(t_bc), X.ctypes.data, W.ctypes.data,
                             psi.ctypes.data, out.ctypes.data, int(out_parity))
    if rc != 0:
        raise ValueError("invalid lattice extents")
    return out


def dslash(dims, t_bc: int, X, W, psi_half: np.ndarray, out_parity: int) -> np.ndarray:
    """Even/odd Dslash on a half-lattice field.

    ``out_parity`` 0 gives D_eo (input on odd sites, output on even sites),
    1 gives D_oe.  ``psi_half`` is (V/2, 3) or (nrhs, V/2, 3).
    """
    psi_half = np.asarray(psi_half)
    if psi_half.ndim == 3:
        return np.stack([dslash(dims, t_bc, X, W, p, out_parity) for p in psi_half])
    full = to_full(psi_half, dims, 1 - out_parity)
    return from_full(dslash_full(dims, t_bc, X, W, full, out_parity), dims, out_parity)


def dslash_at(dims, t_bc: int, X, W, psi_half, in_parity: int, sites_lex) -> np.ndarray:
    """(D psi)(s) at the given lexicographic output sites, psi on ``in_parity``."""
    X = _links(X, dims)
    W = _links(W, dims)
    full = to_full(psi_half, dims, in_parity)
    s = np.ascontiguousarray(sites_lex, dtype=np.int64)
    out = np.empty((len(s), 3), dtype=np.complex128)
    rc = lib().oracle_dslash_sites(_dims_arg(dims), int(t_bc), X.ctypes.data, W.ctypes.data,
                                   full.ctypes.data, s.ctypes.data, len(s), out.ctypes.data)
    if rc != 0:
        raise ValueError("invalid lattice extents")
    return out


@dataclass
class Lattice:
    """A gauge background for the oracle: extents, time BC and the two fields."""
    dims: tuple
    t_bc: int
    X: np.ndarray
    W: np.ndarray

    def D_eo(self, psi_odd):
        return dslash(self.dims, self.t_bc, self.X, self.W, psi_odd, 0)

    def D_oe(self, psi_even):
        return dslash(self.dims, self.t_bc, self.X, self.W, psi_even, 1)

    def M_e(self, mass: float, psi_even, shift: float = 0.0):
        """(m^2 + shift) psi - D_eo D_oe psi on even sites."""
        return (mass * mass + shift) * psi_even - self.D_eo(self.D_oe(psi_even))


def lattice_from(w) -> Lattice:
    return Lattice(tuple(w["dims"]), int(w["t_bc"]), w["fat"], w["naik"])


# ---------------------------------------------------------------------------
# Solvers (Sec. 3.2)
# ---------------------------------------------------------------------------

OK, NOT_CONVERGED, BREAKDOWN = 0, 2, 3


def vdot(a, b) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(np.vdot(np.ravel(a), np.ravel(b)))


def norm(a) -> float:
    return float(np.linalg.norm(np.ravel(a)))


def true_residual(lat: Lattice, mass: float, b, x, shift: float = 0.0) -> float:
    """||b - (M_e + shift) x|| / ||b|| evaluated in FP64."""
    return norm(b - lat.M_e(mass, x, shift)) / norm(b)


@dataclass
class SolveResult:
    x: np.ndarray
    status: int
    iterations: int
    true_residual: float


def cg(lat: Lattice, mass: float, b, tol: float, max_iter: int, x0=None,
       shift: float = 0.0) -> SolveResult:
    """Hestenes-Stiefel CG for (M_e + shift) x = b, stopped on the true residual.

    Textbook CG: q = A p, alpha = rho / Re<p, q>, x += alpha p, r -= alpha q,
    beta = rho'/rho, p = r + beta p.  When the iterated residual meets the
    tolerance the true residual b - A x is formed; if it fails, CG continues
    from it.  A non-positive or non-finite <p, A p> is a breakdown.
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = norm(b)
    if bn == 0.0:
        return SolveResult(np.zeros_like(b), OK, 0, 0.0)
    A = lambda v: lat.M_e(mass, v, shift)  # noqa: E731
    r = b - A(x)
    p = r.copy()
    rho = vdot(r, r).real
    if np.sqrt(rho) <= tol * bn:
        return SolveResult(x, OK, 0, np.sqrt(rho) / bn)
    for k in range(1, max_iter + 1):
        q = A(p)
        pi = vdot(p, q).real
        if not np.isfinite(pi) or pi <= 0.0:
            return SolveResult(x, BREAKDOWN, k, true_residual(lat, mass, b, x, shift))
        alpha = rho / pi
        x = x + alpha * p
        r = r - alpha * q
        rho_new = vdot(r, r).real
        if np.sqrt(rho_new) <= tol * bn:
            r_true = b - A(x)
            rt = norm(r_true)
            if rt <= tol * bn:
                return SolveResult(x, OK, k, rt / bn)
            r = r_true
            rho_new = rt * rt
        beta = rho_new / rho
        p = r + beta * p
        rho = rho_new
    return SolveResult(x, NOT_CONVERGED, max_iter, true_residual(lat, mass, b, x, shift))


def multishift_reference(lat: Lattice, mass: float, shifts, b, tol, max_iter: int):
    """x_k = (M_e + sigma_k)^-1 b, each shift solved independently by plain CG."""
    tols = np.broadcast_to(np.asarray(tol, dtype=np.float64), (len(shifts),))
    return [cg(lat, mass, b, float(t), max_iter, shift=float(s)) for s, t in zip(shifts, tols)]


# ---------------------------------------------------------------------------
# Reduced-precision storage, emulated exactly (inputs rounded, FP64 arithmetic)
# ---------------------------------------------------------------------------
# Storage formats of the reduced-precision path:
#   FP32:   each real and imaginary part rounded to binary32 (nearest-even).
#   R12:    links: rows 0 and 1 rounded as FP64 / FP32, row 2 rebuilt as
#           conj(row0 x row1); colour vectors as FP64 / FP32.
#   W14:    fat links as FP64 / FP32; Naik links: rows 0 and 1 and the factor
#           z (from the FP64 input) rounded as FP64 / FP32, row 2 rebuilt as
#           z conj(row0 x row1); colour vectors as FP64 / FP32.
#   FP16N:  links: each real part rounded once, from binary64, to binary16
#           (nearest-even).
#           colour vectors: per site n = max |component| over the 6 reals,
#           n32 = binary32(n); each real part v stored as binary16(v / n32)
#           (division in FP64, then one rounding to binary16); value = n32 * h.

def quantize_fp32(a):
    a = np.asarray(a)
    return (a.real.astype(np.float32).astype(np.float64)
            + 1j * a.imag.astype(np.float32).astype(np.float64))


def quantize_links_fp16(a):
    a = np.asarray(a)
    f = lambda v: v.astype(np.float16).astype(np.float64)  # noqa: E731
    return f(a.real) + 1j * f(a.imag)


def quantize_field_fp16n(psi):
    """Round a (..., V/2, 3) field to the binary16 + per-site-norm format."""
    psi = np.asarray(psi, dtype=np.complex128)
    n = np.maximum(np.abs(psi.real), np.abs(psi.imag)).max(axis=-1)
    n32 = n.astype(np.float32).astype(np.float64)
    safe = np.where(n32 > 0, n32, 1.0)[..., None]
    f = lambda v: (v / safe).astype(np.float16).astype(np.float64)  # noqa: E731
    out = (f(psi.real) + 1j * f(psi.imag)) * n32[..., None]
    return out


def reconstruct12(U):
    """Keep rows 0 and 1 of each 3x3 matrix and replace row 2 by the complex
    conjugate of their cross product.  For U in SU(3) this returns U (the
    rows are orthonormal and det U = 1, so row 2 = conj(row0 x row1)); any
    other matrix is changed.  This is the reconstruct-12 link compression
    (Sec. 4.4 gauge-field compression types; Sec. 5 notes that the dropped
    entries follow from the SU(3) symmetry)."""
    U = np.array(U, dtype=np.complex128)
    a, b = U[..., 0, :], U[..., 1, :]
    U[..., 2, :] = np.conj(np.cross(a, b))
    return U


def quantize_links_r12(U, prec: str):
    """Reconstruct-12 storage: rows 0 and 1 rounded to `prec` ("fp64" or
    "fp32"), row 2 rebuilt from the rounded rows (in FP64)."""
    U = np.asarray(U, dtype=np.complex128)
    if prec == "fp32":
        U = quantize_fp32(U)
    elif prec != "fp64":
        raise ValueError(prec)
    return reconstruct12(U)


def scaled_row2_factor(U):
    """The complex factor z with row 2 closest to z conj(row0 x row1) in the
    least-squares sense, z = <c, r2> / <c, c> with c = conj(row0 x row1) (0
    where c = 0).  For U in SU(3) z = 1; for U in U(3) z = det U (write
    U = e^{i phi} S with S in SU(3): row 2 = e^{i phi} conj(s0 x s1) and
    conj(u0 x u1) = e^{-2 i phi} conj(s0 x s1)); for a real multiple a V of a
    U(3) matrix z = det V / a."""
    U = np.asarray(U, dtype=np.complex128)
    c = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    cc = np.sum(c.real ** 2 + c.imag ** 2, axis=-1)
    num = np.sum(np.conj(c) * U[..., 2, :], axis=-1)
    d = np.where(cc > 0, cc, 1.0)        # complex / positive real: part by part
    return np.where(cc > 0, num.real / d + 1j * (num.imag / d), 0.0)


def reconstruct_scaled(U, z):
    """Rows 0 and 1 of U kept, row 2 replaced by z conj(row0 x row1)."""
    U = np.array(U, dtype=np.complex128)
    U[..., 2, :] = np.asarray(z)[..., None] * np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    return U


def quantize_links_w14(U, prec: str):
    """The 14-real storage of the Naik links: the factor z of
    scaled_row2_factor formed from the FP64 input, then rows 0 and 1 and z
    rounded to `prec` ("fp64" or "fp32"), row 2 rebuilt from the rounded
    values (in FP64).  Exact (up to that rounding) for SU(3), U(3) and real
    multiples of U(3) matrices, such as the HISQ Naik link c_Naik Y Y Y."""
    U = np.asarray(U, dtype=np.complex128)
    z = scaled_row2_factor(U)
    if prec == "fp32":
        U, z = quantize_fp32(U), quantize_fp32(z)
    elif prec != "fp64":
        raise ValueError(prec)
    return reconstruct_scaled(U, z)


def quantized_lattice(lat: Lattice, prec: str) -> Lattice:
    if prec == "fp64":
        return lat
    if prec == "fp32":
        return Lattice(lat.dims, lat.t_bc, quantize_fp32(lat.X), quantize_fp32(lat.W))
    if prec == "fp16n":
        return Lattice(lat.dims, lat.t_bc, quantize_links_fp16(lat.X), quantize_links_fp16(lat.W))
    if prec in ("fp64r12", "fp32r12"):
        base = prec[:4]
        return Lattice(lat.dims, lat.t_bc, quantize_links_r12(lat.X, base), quantize_links_r12(lat.W, base))
    if prec in ("fp64w14", "fp32w14"):   # fat links in full, Naik links in 14 reals
        base = prec[:4]
        X = lat.X if base == "fp64" else quantize_fp32(lat.X)
        return Lattice(lat.dims, lat.t_bc, X, quantize_links_w14(lat.W, base))
    raise ValueError(prec)


def quantize_field(psi, prec: str):
    if prec in ("fp64r12", "fp32r12", "fp64w14", "fp32w14"):   # colour vectors as in the base precision
        prec = prec[:4]
    if prec == "fp64":
        return np.asarray(psi, dtype=np.complex128)
    if prec == "fp32":
        return quantize_fp32(psi)
    if prec == "fp16n":
        return quantize_field_fp16n(psi)
    raise ValueError(prec)
