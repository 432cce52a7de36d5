"""Thin Python binding of ``libhisq.so`` (the C ABI in ``include/hisq.h``).

Argument marshalling only: torch tensors on the GPU are passed as raw device
pointers, ``torch.cuda.current_stream()`` supplies the ``hipStream_t``, and a
non-OK status raises :class:`HisqError`.  Every computation runs in the HIP
kernels of the library; there is no CPU fallback.  If the library is not
built, :func:`load` raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhisq.so")

HISQ_FP64, HISQ_FP32, HISQ_FP16N, HISQ_FP64R12, HISQ_FP32R12, HISQ_FP64W14, HISQ_FP32W14 = 0, 1, 2, 3, 4, 5, 6
PRECS = {"fp64": HISQ_FP64, "fp32": HISQ_FP32, "fp16n": HISQ_FP16N, "fp64r12": HISQ_FP64R12,
         "fp32r12": HISQ_FP32R12, "fp64w14": HISQ_FP64W14, "fp32w14": HISQ_FP32W14}
HISQ_MAX_RHS = 16
# bytes of the device scratch array behind hisq_apply_m_dot_noalloc
HISQ_NOALLOC_SCRATCH_BYTES = 4 << 20

OK, INVALID_ARG, NOT_CONVERGED, BREAKDOWN, DEVICE, WORKSPACE, UNSUPPORTED = range(7)


class HisqError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class hisq_lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("t_bc", ctypes.c_int32)]


class hisq_dslash_shape(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("nin", ctypes.c_int32), ("block", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32)]

    def as_tuple(self):
        return (self.variant, self.nin, self.block, self.xcd_remap)


class hisq_problem(ctypes.Structure):
    _fields_ = [("lat", hisq_lattice), ("mass", ctypes.c_double), ("links_f64", ctypes.c_void_p),
                ("links_inner", ctypes.c_void_p), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("tol", ctypes.c_double)]


class hisq_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
                ("true_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("shared_iterations", ctypes.c_int32), ("refine_iterations", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = ctypes.c_void_p
_LAT = ctypes.POINTER(hisq_lattice)

# name -> (restype, argtypes)
_SIGS = {
    "hisq_context_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32]),
    "hisq_context_destroy": (None, [_vp]),
    "hisq_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "hisq_last_error": (ctypes.c_char_p, []),
    "hisq_links_bytes": (ctypes.c_size_t, [_LAT, ctypes.c_int]),
    "hisq_field_bytes": (ctypes.c_size_t, [_LAT, ctypes.c_int, ctypes.c_int32]),
    "hisq_pack_links": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "hisq_unpack_links": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "hisq_pack_field": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, ctypes.c_int32, _vp, _vp, _vp]),
    "hisq_unpack_field": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, ctypes.c_int32, _vp, _vp, _vp]),
    "hisq_dslash": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, ctypes.c_int32, _vp, _vp, _vp,
                                   ctypes.c_int32, _vp]),
    "hisq_apply_m": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, ctypes.c_double, _vp, _vp, _vp, _vp,
                                    ctypes.c_int32, _vp]),
    "hisq_apply_m_dot_workspace_bytes": (ctypes.c_size_t, [_LAT, ctypes.c_int32]),
    "hisq_apply_m_dot": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, ctypes.c_int, ctypes.c_double, _vp, _vp, _vp, _vp,
                                        ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp]),
    "hisq_apply_m_dot_noalloc": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, ctypes.c_int, ctypes.c_double, _vp, _vp,
                                                _vp, _vp, ctypes.c_int32, _vp, _vp]),
    "hisq_stream_copy": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "hisq_stream_read_sink_words": (ctypes.c_size_t, [ctypes.c_size_t]),
    "hisq_stream_read": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp, _vp]),
    "hisq_smear_workspace_bytes": (ctypes.c_size_t, [_LAT]),
    "hisq_smear_links": (ctypes.c_int, [_vp, _LAT, _vp, ctypes.c_double, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "hisq_tune_dslash": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, ctypes.c_int32, _vp, _vp, _vp, _vp]),
    "hisq_get_dslash_shape": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, ctypes.c_int32,
                                             ctypes.POINTER(hisq_dslash_shape)]),
    "hisq_set_dslash_shape": (ctypes.c_int, [_vp, _LAT, ctypes.c_int, ctypes.c_int32,
                                             ctypes.POINTER(hisq_dslash_shape)]),
    "hisq_cg_workspace_bytes": (ctypes.c_size_t, [_LAT, ctypes.c_int, ctypes.c_int32, ctypes.c_int32]),
    "hisq_cg": (ctypes.c_int, [_vp, _LAT, ctypes.c_double, _vp, _vp, ctypes.c_int, ctypes.c_int32, _vp, _vp,
                               ctypes.c_double, ctypes.c_int32, _vp, ctypes.c_size_t,
                               ctypes.POINTER(hisq_solve_info), _vp]),
    "hisq_chiral_condensate": (ctypes.c_int, [_vp, _LAT, ctypes.c_double, _vp, _vp, ctypes.c_int, ctypes.c_int32,
                                              _vp, _vp, ctypes.c_double, ctypes.c_int32, _vp, ctypes.c_size_t,
                                              _vp, _vp, _vp, _vp, _vp]),
    "hisq_multishift_cg": (ctypes.c_int, [_vp, _LAT, ctypes.c_double, _vp, _vp, ctypes.c_int, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double), _vp, ctypes.POINTER(_vp),
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int32, _vp, ctypes.c_size_t,
                                          ctypes.POINTER(hisq_solve_info), _vp]),
    "hisq_multishift_krylov": (ctypes.c_int, [_vp, _LAT, ctypes.c_double, _vp, _vp, ctypes.c_int, ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_double), _vp, ctypes.POINTER(_vp),
                                              ctypes.POINTER(ctypes.c_double), ctypes.c_int32, _vp,
                                              ctypes.c_size_t, ctypes.POINTER(hisq_solve_info), _vp]),
    "hisq_cg_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.POINTER(hisq_problem),
                                                        ctypes.c_int]),
    "hisq_cg_batch": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(hisq_problem), ctypes.c_int,
                                     ctypes.c_int32, _vp, ctypes.c_size_t, ctypes.POINTER(hisq_solve_info),
                                     ctypes.POINTER(ctypes.c_double), _vp]),
    "hisq_ptc_workspace_bytes": (ctypes.c_size_t, [_LAT]),
    "hisq_ptc_forward": (ctypes.c_int, [_vp, _LAT, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "hisq_ptc_backward": (ctypes.c_int, [_vp, _LAT, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "hisq_ptc_adam_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp]),
    "hisq_ptc_train_step": (ctypes.c_int, [_vp, _LAT, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                           ctypes.c_int32,
                                           _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.POINTER(ctypes.c_double), _vp,
                                           ctypes.c_size_t, _vp]),
    "hisq_fcg_workspace_bytes": (ctypes.c_size_t, [_LAT]),
    "hisq_fcg": (ctypes.c_int, [_vp, _LAT, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, ctypes.c_double,
                                ctypes.c_int32, _vp, ctypes.c_size_t, ctypes.POINTER(hisq_solve_info), _vp]),
}


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it is missing: no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def declared_symbols():
    return list(_SIGS)


def _check(status: int, where: str):
    if status != OK:
        lib = load()
        detail = lib.hisq_last_error().decode() or lib.hisq_status_string(status).decode()
        raise HisqError(status, where, detail)


def lattice(dims, t_bc: int) -> hisq_lattice:
    lat = hisq_lattice()
    for k in range(4):
        lat.dims[k] = int(dims[k])
    lat.t_bc = int(t_bc)
    return lat


def _prec(p) -> int:
    return PRECS[p] if isinstance(p, str) else int(p)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def _ptr(t: torch.Tensor | None, name: str, nbytes: int | None = None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if nbytes is not None and t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name} holds {t.numel() * t.element_size()} bytes, needs {nbytes}")
    return _vp(t.data_ptr())


class Context:
    """Owns a hisq_context (device + autotune cache)."""

    def __init__(self, device: int = 0):
        h = _vp()
        _check(load().hisq_context_create(ctypes.byref(h), int(device)), "hisq_context_create")
        self.handle = h

    def close(self):
        if self.handle:
            load().hisq_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ctx(ctx):
    return None if ctx is None else ctx.handle


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def hisq_links_bytes(lat: hisq_lattice, prec) -> int:
    return int(load().hisq_links_bytes(ctypes.byref(lat), _prec(prec)))


def hisq_field_bytes(lat: hisq_lattice, prec, nrhs: int = 1) -> int:
    return int(load().hisq_field_bytes(ctypes.byref(lat), _prec(prec), int(nrhs)))


def empty_links(lat, prec, device="cuda") -> torch.Tensor:
    return torch.empty(hisq_links_bytes(lat, prec), dtype=torch.uint8, device=device)


def packed_bytes(lat, prec, nrhs: int) -> int:
    """Bytes of nrhs packed fields stored as groups of HISQ_MAX_RHS columns
    one after another (the last group holding the rest)."""
    full, rest = divmod(int(nrhs), HISQ_MAX_RHS)
    return full * hisq_field_bytes(lat, prec, HISQ_MAX_RHS) + (hisq_field_bytes(lat, prec, rest) if rest else 0)


def empty_field(lat, prec, nrhs: int = 1, device="cuda") -> torch.Tensor:
    """Room for nrhs packed fields (any number, as groups of HISQ_MAX_RHS
    columns; the C calls take at most HISQ_MAX_RHS at a time)."""
    return torch.empty(packed_bytes(lat, prec, nrhs), dtype=torch.uint8, device=device)


def hisq_pack_links(lat, prec, fat_c128: torch.Tensor, naik_c128: torch.Tensor, packed: torch.Tensor,
                    ctx=None, stream=None):
    vol = 1
    for d in lat.dims:
        vol *= d
    n = 4 * vol * 9 * 16
    _check(load().hisq_pack_links(_ctx(ctx), ctypes.byref(lat), _prec(prec),
                                  _ptr(fat_c128, "fat_c128", n), _ptr(naik_c128, "naik_c128", n),
                                  _ptr(packed, "packed", hisq_links_bytes(lat, prec)), _stream(stream)),
           "hisq_pack_links")


def hisq_unpack_links(lat, prec, packed: torch.Tensor, fat_c128: torch.Tensor, naik_c128: torch.Tensor,
                      ctx=None, stream=None):
    vol = 1
    for d in lat.dims:
        vol *= d
    n = 4 * vol * 9 * 16
    _check(load().hisq_unpack_links(_ctx(ctx), ctypes.byref(lat), _prec(prec),
                                    _ptr(packed, "packed", hisq_links_bytes(lat, prec)),
                                    _ptr(fat_c128, "fat_c128", n), _ptr(naik_c128, "naik_c128", n),
                                    _stream(stream)), "hisq_unpack_links")


def _half_bytes(lat, nrhs):
    vol = 1
    for d in lat.dims:
        vol *= d
    return nrhs * (vol // 2) * 3 * 16


def hisq_pack_field(lat, prec, nrhs: int, half_c128: torch.Tensor, packed: torch.Tensor,
                    ctx=None, stream=None):
    _check(load().hisq_pack_field(_ctx(ctx), ctypes.byref(lat), _prec(prec), int(nrhs),
                                  _ptr(half_c128, "half_c128", _half_bytes(lat, nrhs)),
                                  _ptr(packed, "packed", hisq_field_bytes(lat, prec, nrhs)),
                                  _stream(stream)), "hisq_pack_field")


def hisq_unpack_field(lat, prec, nrhs: int, packed: torch.Tensor, half_c128: torch.Tensor,
                      ctx=None, stream=None):
    _check(load().hisq_unpack_field(_ctx(ctx), ctypes.byref(lat), _prec(prec), int(nrhs),
                                    _ptr(packed, "packed", hisq_field_bytes(lat, prec, nrhs)),
                                    _ptr(half_c128, "half_c128", _half_bytes(lat, nrhs)),
                                    _stream(stream)), "hisq_unpack_field")


def hisq_dslash(lat, prec, out_parity: int, links, inp, out, nrhs: int = 1, ctx=None, stream=None):
    fb = hisq_field_bytes(lat, prec, nrhs)
    _check(load().hisq_dslash(_ctx(ctx), ctypes.byref(lat), _prec(prec), int(out_parity),
                              _ptr(links, "links", hisq_links_bytes(lat, prec)),
                              _ptr(inp, "in", fb), _ptr(out, "out", fb), int(nrhs), _stream(stream)),
           "hisq_dslash")


def hisq_apply_m(lat, prec, mass: float, links, in_even, out_even, tmp_odd, nrhs: int = 1,
                 ctx=None, stream=None):
    fb = hisq_field_bytes(lat, prec, nrhs)
    _check(load().hisq_apply_m(_ctx(ctx), ctypes.byref(lat), _prec(prec), float(mass),
                               _ptr(links, "links", hisq_links_bytes(lat, prec)),
                               _ptr(in_even, "in_even", fb), _ptr(out_even, "out_even", fb),
                               _ptr(tmp_odd, "tmp_odd", fb), int(nrhs), _stream(stream)),
           "hisq_apply_m")


def hisq_apply_m_dot_workspace_bytes(lat, nrhs: int = 1) -> int:
    return int(load().hisq_apply_m_dot_workspace_bytes(ctypes.byref(lat), int(nrhs)))


def hisq_apply_m_dot(lat, link_prec, field_prec, mass: float, links, in_even, out_even, tmp_odd, dot_out, ws,
                     nrhs: int = 1, ctx=None, stream=None):
    """out_even = M_e in_even and dot_out[r] = Re <in_r, out_r> (dot_out: a
    float64 GPU tensor of nrhs entries)."""
    fb = hisq_field_bytes(lat, field_prec, nrhs)
    _check(load().hisq_apply_m_dot(_ctx(ctx), ctypes.byref(lat), _prec(link_prec), _prec(field_prec), float(mass),
                                   _ptr(links, "links", hisq_links_bytes(lat, link_prec)),
                                   _ptr(in_even, "in_even", fb), _ptr(out_even, "out_even", fb),
                                   _ptr(tmp_odd, "tmp_odd", fb), int(nrhs), _ptr(dot_out, "dot_out", 8 * int(nrhs)),
                                   _ptr(ws, "ws"), ctypes.c_size_t(ws.numel() * ws.element_size()),
                                   _stream(stream)), "hisq_apply_m_dot")


def hisq_apply_m_dot_noalloc(lat, link_prec, field_prec, mass: float, links, in_even, out_even, tmp_odd, dot_out,
                             nrhs: int = 1, ctx=None, stream=None):
    """hisq_apply_m_dot with its block partials in the library's static
    device scratch (no workspace argument; allocates nothing)."""
    fb = hisq_field_bytes(lat, field_prec, nrhs)
    _check(load().hisq_apply_m_dot_noalloc(_ctx(ctx), ctypes.byref(lat), _prec(link_prec), _prec(field_prec),
                                           float(mass), _ptr(links, "links", hisq_links_bytes(lat, link_prec)),
                                           _ptr(in_even, "in_even", fb), _ptr(out_even, "out_even", fb),
                                           _ptr(tmp_odd, "tmp_odd", fb), int(nrhs),
                                           _ptr(dot_out, "dot_out", 8 * int(nrhs)), _stream(stream)),
           "hisq_apply_m_dot_noalloc")


def hisq_stream_copy(src, dst, nbytes: int | None = None, ctx=None, stream=None):
    """dst = src (first nbytes bytes, default all of src) with the library's
    streaming copy kernel: the bandwidth reference of the benchmark."""
    n = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    _check(load().hisq_stream_copy(_ctx(ctx), _ptr(src, "src", n), _ptr(dst, "dst", n), n, _stream(stream)),
           "hisq_stream_copy")


def hisq_stream_read_sink_words(nbytes: int) -> int:
    return int(load().hisq_stream_read_sink_words(int(nbytes)))


def hisq_stream_read(src, sink, nbytes: int | None = None, ctx=None, stream=None):
    """Reads the first nbytes bytes of src (default all) with the library's
    read-only streaming kernel; sink (uint32/int32 device tensor of
    hisq_stream_read_sink_words(nbytes) words) receives one XOR per 16 KiB."""
    n = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    words = hisq_stream_read_sink_words(n)
    _check(load().hisq_stream_read(_ctx(ctx), _ptr(src, "src", n), n, _ptr(sink, "sink", 4 * words),
                                   _stream(stream)), "hisq_stream_read")


def hisq_smear_workspace_bytes(lat) -> int:
    return int(load().hisq_smear_workspace_bytes(ctypes.byref(lat)))


def hisq_smear_links(lat, thin_c128, fat_c128, naik_c128, ws, naik_eps: float = 0.0, ctx=None, stream=None):
    """HISQ fat and Naik links (canonical complex128 layout) from thin links."""
    n = 1
    for d in lat.dims:
        n *= d
    n *= 4 * 9 * 16
    _check(load().hisq_smear_links(_ctx(ctx), ctypes.byref(lat), _ptr(thin_c128, "thin_c128", n), float(naik_eps),
                                   _ptr(fat_c128, "fat_c128", n), _ptr(naik_c128, "naik_c128", n),
                                   _ptr(ws, "ws", hisq_smear_workspace_bytes(lat)), ctypes.c_size_t(ws.numel()),
                                   _stream(stream)), "hisq_smear_links")


def hisq_tune_dslash(lat, prec, nrhs: int, links, inp, out, ctx, stream=None):
    fb = hisq_field_bytes(lat, prec, nrhs)
    _check(load().hisq_tune_dslash(_ctx(ctx), ctypes.byref(lat), _prec(prec), int(nrhs),
                                   _ptr(links, "links", hisq_links_bytes(lat, prec)),
                                   _ptr(inp, "in", fb), _ptr(out, "out", fb), _stream(stream)),
           "hisq_tune_dslash")


def hisq_get_dslash_shape(lat, prec, nrhs: int = 1, ctx=None):
    sh = hisq_dslash_shape()
    _check(load().hisq_get_dslash_shape(_ctx(ctx), ctypes.byref(lat), _prec(prec), int(nrhs),
                                        ctypes.byref(sh)), "hisq_get_dslash_shape")
    return sh.as_tuple()


def hisq_set_dslash_shape(lat, prec, nrhs: int, shape, ctx):
    sh = hisq_dslash_shape(*[int(v) for v in shape])
    _check(load().hisq_set_dslash_shape(_ctx(ctx), ctypes.byref(lat), _prec(prec), int(nrhs),
                                        ctypes.byref(sh)), "hisq_set_dslash_shape")


def hisq_cg_workspace_bytes(lat, inner, nrhs: int = 1, nshift: int = 0) -> int:
    return int(load().hisq_cg_workspace_bytes(ctypes.byref(lat), _prec(inner), int(nrhs), int(nshift)))


def empty_workspace(nbytes: int) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


def hisq_cg(lat, mass: float, links_f64, links_inner, inner, nrhs: int, b, x, tol: float, max_iter: int,
            ws, ctx=None, stream=None, check: bool = True):
    """Returns (status, [info dict per right-hand side]); raises on errors other
    than NOT_CONVERGED / BREAKDOWN unless check is False."""
    info = (hisq_solve_info * int(nrhs))()
    fb = hisq_field_bytes(lat, "fp64", nrhs)
    st = load().hisq_cg(_ctx(ctx), ctypes.byref(lat), float(mass),
                        _ptr(links_f64, "links_f64", hisq_links_bytes(lat, "fp64")),
                        None if links_inner is None else _ptr(links_inner, "links_inner",
                                                              hisq_links_bytes(lat, inner)),
                        _prec(inner), int(nrhs), _ptr(b, "b", fb), _ptr(x, "x", fb), float(tol),
                        int(max_iter), _ptr(ws, "ws"), ctypes.c_size_t(ws.numel()), info, _stream(stream))
    if check and st not in (OK, NOT_CONVERGED, BREAKDOWN):
        _check(st, "hisq_cg")
    return st, [info[k].as_dict() for k in range(int(nrhs))]


def hisq_chiral_condensate(lat, mass: float, links_f64, links_inner, inner, nnoise: int, noise, x, tol: float,
                           max_iter: int, ws, ctx=None, stream=None, check: bool = True):
    """Returns (status, pbp, err, samples list, [info dict per noise vector])."""
    fb = hisq_field_bytes(lat, "fp64", 1)
    smp = (ctypes.c_double * int(nnoise))()
    info = (hisq_solve_info * int(nnoise))()
    pbp, err = ctypes.c_double(), ctypes.c_double()
    lin = None if links_inner is None else _ptr(links_inner, "links_inner", hisq_links_bytes(lat, inner))
    st = load().hisq_chiral_condensate(_ctx(ctx), ctypes.byref(lat), float(mass),
                                       _ptr(links_f64, "links_f64", hisq_links_bytes(lat, "fp64")), lin,
                                       _prec(inner), int(nnoise), _ptr(noise, "noise", nnoise * fb),
                                       _ptr(x, "x", nnoise * fb), float(tol), int(max_iter),
                                       _ptr(ws, "ws"), ctypes.c_size_t(ws.numel()), smp, ctypes.byref(pbp),
                                       ctypes.byref(err), info, _stream(stream))
    if check and st not in (OK, NOT_CONVERGED, BREAKDOWN):
        _check(st, "hisq_chiral_condensate")
    return st, pbp.value, err.value, list(smp), [info[k].as_dict() for k in range(int(nnoise))]


def hisq_multishift_cg(lat, mass: float, links_f64, links_inner, inner, shifts, b, xs, tol, max_iter: int,
                       ws, ctx=None, stream=None, check: bool = True):
    """xs: list of packed FP64 fields, one per shift.  tol: scalar or per shift."""
    n = len(shifts)
    sh = (ctypes.c_double * n)(*[float(v) for v in shifts])
    tols = [float(tol)] * n if not hasattr(tol, "__len__") else [float(v) for v in tol]
    tl = (ctypes.c_double * n)(*tols)
    fb = hisq_field_bytes(lat, "fp64", 1)
    xp = (_vp * n)(*[_ptr(xk, f"x[{k}]", fb) for k, xk in enumerate(xs)])
    info = (hisq_solve_info * n)()
    st = load().hisq_multishift_cg(_ctx(ctx), ctypes.byref(lat), float(mass),
                                   _ptr(links_f64, "links_f64", hisq_links_bytes(lat, "fp64")),
                                   None if links_inner is None else _ptr(links_inner, "links_inner",
                                                                         hisq_links_bytes(lat, inner)),
                                   _prec(inner), n, sh, _ptr(b, "b", fb), xp, tl, int(max_iter),
                                   _ptr(ws, "ws"), ctypes.c_size_t(ws.numel()), info, _stream(stream))
    if check and st not in (OK, NOT_CONVERGED, BREAKDOWN):
        _check(st, "hisq_multishift_cg")
    return st, [info[k].as_dict() for k in range(n)]


def hisq_multishift_krylov(lat, mass: float, links_f64, links_inner, inner, shifts, b, xs, tol, max_iter: int,
                           ws, ctx=None, stream=None, check: bool = True):
    """The shared Krylov phase of the multi-shift solver alone (no refinement):
    returns (status, [info dict per shift])."""
    n = len(shifts)
    sh = (ctypes.c_double * n)(*[float(v) for v in shifts])
    tols = [float(tol)] * n if not hasattr(tol, "__len__") else [float(v) for v in tol]
    tl = (ctypes.c_double * n)(*tols)
    fb = hisq_field_bytes(lat, "fp64", 1)
    xp = (_vp * n)(*[_ptr(xk, f"x[{k}]", fb) for k, xk in enumerate(xs)])
    info = (hisq_solve_info * n)()
    st = load().hisq_multishift_krylov(_ctx(ctx), ctypes.byref(lat), float(mass),
                                       _ptr(links_f64, "links_f64", hisq_links_bytes(lat, "fp64")),
                                       None if links_inner is None else _ptr(links_inner, "links_inner",
                                                                             hisq_links_bytes(lat, inner)),
                                       _prec(inner), n, sh, _ptr(b, "b", fb), xp, tl, int(max_iter),
                                       _ptr(ws, "ws"), ctypes.c_size_t(ws.numel()), info, _stream(stream))
    if check and st not in (OK, NOT_CONVERGED, BREAKDOWN):
        _check(st, "hisq_multishift_krylov")
    return st, [info[k].as_dict() for k in range(n)]


def make_problems(items):
    """items: list of dicts with lat, mass, links_f64, links_inner, b, x, tol
    (tensors); returns the ctypes array (keeps no references: hold the tensors)."""
    arr = (hisq_problem * len(items))()
    for k, it in enumerate(items):
        lat = it["lat"]
        fb = hisq_field_bytes(lat, "fp64", 1)
        arr[k].lat = lat
        arr[k].mass = float(it["mass"])
        arr[k].links_f64 = _ptr(it["links_f64"], "links_f64", hisq_links_bytes(lat, "fp64"))
        li = it.get("links_inner")
        arr[k].links_inner = None if li is None else _ptr(li, "links_inner")
        arr[k].b = _ptr(it["b"], "b", fb)
        arr[k].x = _ptr(it["x"], "x", fb)
        arr[k].tol = float(it["tol"])
    return arr


def hisq_cg_batch_workspace_bytes(problems, inner) -> int:
    return int(load().hisq_cg_batch_workspace_bytes(len(problems), problems, _prec(inner)))


def hisq_cg_batch(problems, inner, max_iter: int, ws, ctx=None, stream=None, check: bool = True):
    """problems: array from make_problems.  Returns (status, infos, latencies)."""
    n = len(problems)
    info = (hisq_solve_info * n)()
    lat_s = (ctypes.c_double * n)()
    st = load().hisq_cg_batch(_ctx(ctx), n, problems, _prec(inner), int(max_iter), _ptr(ws, "ws"),
                              ctypes.c_size_t(ws.numel()), info, lat_s, _stream(stream))
    if check and st not in (OK, NOT_CONVERGED, BREAKDOWN):
        _check(st, "hisq_cg_batch")
    return st, [info[k].as_dict() for k in range(n)], [lat_s[k] for k in range(n)]


HISQ_PTC_NWEIGHTS = 720


def hisq_ptc_workspace_bytes(lat) -> int:
    return int(load().hisq_ptc_workspace_bytes(ctypes.byref(lat)))


def hisq_ptc_forward(lat, links_f32, weights, in_even, out_even, ws, ctx=None, stream=None):
    fb = hisq_field_bytes(lat, "fp32", 1)
    _check(load().hisq_ptc_forward(_ctx(ctx), ctypes.byref(lat), _ptr(links_f32, "links_f32",
                                                                      hisq_links_bytes(lat, "fp32")),
                                   _ptr(weights, "weights", HISQ_PTC_NWEIGHTS * 8), _ptr(in_even, "in_even", fb),
                                   _ptr(out_even, "out_even", fb), _ptr(ws, "ws"), ctypes.c_size_t(ws.numel()),
                                   _stream(stream)), "hisq_ptc_forward")


def hisq_ptc_backward(lat, links_f32, weights, g_out_even, g_in_even, grad, ws, ctx=None, stream=None):
    fb = hisq_field_bytes(lat, "fp32", 1)
    _check(load().hisq_ptc_backward(_ctx(ctx), ctypes.byref(lat),
                                    _ptr(links_f32, "links_f32", hisq_links_bytes(lat, "fp32")),
                                    _ptr(weights, "weights", HISQ_PTC_NWEIGHTS * 8),
                                    _ptr(g_out_even, "g_out_even", fb), _ptr(g_in_even, "g_in_even", fb),
                                    _ptr(grad, "grad", HISQ_PTC_NWEIGHTS * 16), _ptr(ws, "ws"),
                                    ctypes.c_size_t(ws.numel()), _stream(stream)), "hisq_ptc_backward")


def hisq_ptc_adam_step(w_master, w_f32, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                       ctx=None, stream=None):
    n16 = HISQ_PTC_NWEIGHTS * 16
    _check(load().hisq_ptc_adam_step(_ctx(ctx), _ptr(w_master, "w_master", n16),
                                     _ptr(w_f32, "w_f32", HISQ_PTC_NWEIGHTS * 8), _ptr(grad, "grad", n16),
                                     _ptr(m, "m", n16), _ptr(v, "v", n16), int(step), float(lr), float(beta1),
                                     float(beta2), float(eps), _stream(stream)), "hisq_ptc_adam_step")


def hisq_ptc_train_step(lat, mass, links_f32, w_master, w_f32, m, v, step, batch, src_f32, sol_f64, ws,
                        lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, ctx=None, stream=None) -> float:
    n16 = HISQ_PTC_NWEIGHTS * 16
    loss = ctypes.c_double()
    _check(load().hisq_ptc_train_step(_ctx(ctx), ctypes.byref(lat), float(mass),
                                      _ptr(links_f32, "links_f32", hisq_links_bytes(lat, "fp32")),
                                      _ptr(w_master, "w_master", n16), _ptr(w_f32, "w_f32", HISQ_PTC_NWEIGHTS * 8),
                                      _ptr(m, "m", n16), _ptr(v, "v", n16), int(step), int(batch),
                                      _ptr(src_f32, "src_f32", hisq_field_bytes(lat, "fp32", batch)),
                                      _ptr(sol_f64, "sol_f64", hisq_field_bytes(lat, "fp64", batch)),
                                      float(lr), float(beta1), float(beta2), float(eps), ctypes.byref(loss),
                                      _ptr(ws, "ws"), ctypes.c_size_t(ws.numel()), _stream(stream)),
           "hisq_ptc_train_step")
    return loss.value


def hisq_fcg_workspace_bytes(lat) -> int:
    return int(load().hisq_fcg_workspace_bytes(ctypes.byref(lat)))


def hisq_fcg(lat, mass, links_f64, links_f32, weights, b, x, tol, max_iter, ws, ctx=None, stream=None,
             check: bool = True):
    info = hisq_solve_info()
    fb = hisq_field_bytes(lat, "fp64", 1)
    st = load().hisq_fcg(_ctx(ctx), ctypes.byref(lat), float(mass),
                         _ptr(links_f64, "links_f64", hisq_links_bytes(lat, "fp64")),
                         _ptr(links_f32, "links_f32", hisq_links_bytes(lat, "fp32")),
                         _ptr(weights, "weights", HISQ_PTC_NWEIGHTS * 8), _ptr(b, "b", fb), _ptr(x, "x", fb),
                         float(tol), int(max_iter), _ptr(ws, "ws"), ctypes.c_size_t(ws.numel()),
                         ctypes.byref(info), _stream(stream))
    if check and st not in (OK, NOT_CONVERGED, BREAKDOWN):
        _check(st, "hisq_fcg")
    return st, info.as_dict()


def weights_to_device(ws_list):
    """Oracle-layout weights (list of [c_out][c_in][9] complex arrays) ->
    (FP64 master double2 tensor, FP32 float2 tensor) on the GPU."""
    import numpy as np
    flat = np.concatenate([np.asarray(w, dtype=np.complex128).ravel() for w in ws_list])
    assert flat.size == HISQ_PTC_NWEIGHTS
    master = torch.from_numpy(flat.view(np.float64).copy()).cuda()
    f32 = master.to(torch.float32)
    return master, f32


def weights_from_device(master):
    import numpy as np
    flat = master.cpu().numpy().view(np.complex128)
    shapes = [(8, 1, 9), (8, 8, 9), (1, 8, 9)]
    out, k = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        out.append(flat[k:k + n].reshape(sh))
        k += n
    return out


# ---------------------------------------------------------------------------
# Conveniences built only from the entry points above
# ---------------------------------------------------------------------------

def to_device_c128(a) -> torch.Tensor:
    """Host complex array -> contiguous complex128 GPU tensor."""
    return torch.as_tensor(a, dtype=torch.complex128).contiguous().cuda()


def pack_links_from_host(lat, prec, fat, naik, ctx=None) -> torch.Tensor:
    packed = empty_links(lat, prec)
    f, w = to_device_c128(fat), to_device_c128(naik)
    hisq_pack_links(lat, prec, f, w, packed, ctx=ctx)
    del f, w
    return packed


def pack_field_from_host(lat, prec, half, ctx=None) -> torch.Tensor:
    """Any number of fields, packed in groups of HISQ_MAX_RHS columns one
    after another (packed_bytes)."""
    half = torch.as_tensor(half, dtype=torch.complex128)
    if half.dim() == 2:
        half = half[None]
    nrhs = half.shape[0]
    packed = torch.empty(packed_bytes(lat, prec, nrhs), dtype=torch.uint8, device="cuda")
    for k in range(0, nrhs, HISQ_MAX_RHS):
        n = min(HISQ_MAX_RHS, nrhs - k)
        o = packed_bytes(lat, prec, k)
        hisq_pack_field(lat, prec, n, half[k:k + n].contiguous().cuda(),
                        packed[o:o + hisq_field_bytes(lat, prec, n)], ctx=ctx)
    return packed


def unpack_field_to_host(lat, prec, packed, nrhs: int = 1, ctx=None):
    vol = 1
    for d in lat.dims:
        vol *= d
    out = torch.empty((nrhs, vol // 2, 3), dtype=torch.complex128, device="cuda")
    for k in range(0, nrhs, HISQ_MAX_RHS):
        n = min(HISQ_MAX_RHS, nrhs - k)
        o = packed_bytes(lat, prec, k)
        hisq_unpack_field(lat, prec, n, packed[o:o + hisq_field_bytes(lat, prec, n)], out[k:k + n], ctx=ctx)
    torch.cuda.synchronize()
    return out.cpu().numpy()
