"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments on the host before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hisq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hisq_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2306_01098_amd import hisq as h
    return h.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_2306_01098_amd import hisq as h
    assert sorted(h.declared_symbols()) == declared_functions()


def test_status_strings(lib):
    from paper_2306_01098_amd import hisq as h
    for s in range(7):
        assert lib.hisq_status_string(s)
    assert lib.hisq_status_string(h.NOT_CONVERGED) == b"not converged"


@pytest.mark.parametrize("dims,t_bc", [((4, 4, 4, 5), 1), ((2, 4, 4, 4), 1), ((4, 4, 4, 4), 0),
                                      ((0, 4, 4, 4), -1)])
def test_invalid_lattice_rejected(lib, dims, t_bc):
    from paper_2306_01098_amd import hisq as h
    lat = h.lattice(dims, t_bc)
    assert h.hisq_links_bytes(lat, "fp64") == 0
    st = lib.hisq_dslash(None, ctypes.byref(lat), 0, 0, ctypes.c_void_p(16), ctypes.c_void_p(32),
                         ctypes.c_void_p(48), 1, None)
    assert st == h.INVALID_ARG
    assert lib.hisq_last_error()


def test_sizes(lib):
    from paper_2306_01098_amd import hisq as h
    lat = h.lattice((32, 32, 32, 8), -1)
    V = 32 ** 3 * 8
    assert h.hisq_links_bytes(lat, "fp64") == 2 * 4 * V * 18 * 8 == 301989888
    assert h.hisq_links_bytes(lat, "fp32") == 2 * 4 * V * 18 * 4
    assert h.hisq_links_bytes(lat, "fp16n") == 2 * 4 * V * 18 * 2
    assert h.hisq_field_bytes(lat, "fp64", 3) == 3 * (V // 2) * 48
    assert h.hisq_field_bytes(lat, "fp16n", 1) == (V // 2) * 16
    assert h.hisq_field_bytes(lat, "fp64", 17) == 0
    assert h.hisq_field_bytes(lat, "fp64", 0) == 0
    # reconstruct-12: rows 0 and 1 of each link; fields as the base precision
    assert h.hisq_links_bytes(lat, "fp64r12") == 2 * 4 * V * 12 * 8
    assert h.hisq_links_bytes(lat, "fp32r12") == 2 * 4 * V * 12 * 4
    assert h.hisq_field_bytes(lat, "fp64r12", 2) == h.hisq_field_bytes(lat, "fp64", 2)
    assert h.hisq_field_bytes(lat, "fp32r12", 2) == h.hisq_field_bytes(lat, "fp32", 2)
    # W14: fat links in full (18 reals), Naik links in 14
    assert h.hisq_links_bytes(lat, "fp64w14") == 4 * V * (18 + 14) * 8
    assert h.hisq_links_bytes(lat, "fp32w14") == 4 * V * (18 + 14) * 4
    assert h.hisq_field_bytes(lat, "fp64w14", 2) == h.hisq_field_bytes(lat, "fp64", 2)
    assert h.hisq_field_bytes(lat, "fp32w14", 2) == h.hisq_field_bytes(lat, "fp32", 2)
    assert h.hisq_links_bytes(lat, 7) == 0


def test_dslash_argument_checks(lib):
    from paper_2306_01098_amd import hisq as h
    lat = ctypes.byref(h.lattice((4, 4, 4, 4), 1))
    p = ctypes.c_void_p
    # bad parity, NULL pointer, aliasing, bad nrhs, bad precision
    assert lib.hisq_dslash(None, lat, 0, 2, p(16), p(32), p(48), 1, None) == h.INVALID_ARG
    assert lib.hisq_dslash(None, lat, 0, 0, None, p(32), p(48), 1, None) == h.INVALID_ARG
    assert lib.hisq_dslash(None, lat, 0, 0, p(16), p(32), p(32), 1, None) == h.INVALID_ARG
    assert lib.hisq_dslash(None, lat, 0, 0, p(16), p(32), p(48), 0, None) == h.INVALID_ARG
    assert lib.hisq_dslash(None, lat, 7, 0, p(16), p(32), p(48), 1, None) == h.INVALID_ARG
    assert lib.hisq_apply_m(None, lat, 0, 0.0, p(16), p(32), p(48), p(64), 1, None) == h.INVALID_ARG
    assert b"mass" in lib.hisq_last_error()


def test_solver_argument_checks_on_host(lib):
    """Invalid solver arguments are rejected before any HIP call."""
    from paper_2306_01098_amd import hisq as h
    lat = h.lattice((4, 4, 4, 4), -1)
    p = ctypes.c_void_p
    info = (h.hisq_solve_info * 2)()
    # tol outside (0, 1), mass 0, NULL b, aliasing b and x, bad nrhs
    assert lib.hisq_cg(None, ctypes.byref(lat), 0.1, p(16), None, 0, 1, p(32), p(48), 0.0, 10, p(64), 1 << 20,
                       info, None) == h.INVALID_ARG
    assert lib.hisq_cg(None, ctypes.byref(lat), 0.0, p(16), None, 0, 1, p(32), p(48), 1e-8, 10, p(64), 1 << 20,
                       info, None) == h.INVALID_ARG
    assert lib.hisq_cg(None, ctypes.byref(lat), 0.1, p(16), None, 0, 1, None, p(48), 1e-8, 10, p(64), 1 << 20,
                       info, None) == h.INVALID_ARG
    assert lib.hisq_cg(None, ctypes.byref(lat), 0.1, p(16), None, 0, 1, p(32), p(32), 1e-8, 10, p(64), 1 << 20,
                       info, None) == h.INVALID_ARG
    assert lib.hisq_cg(None, ctypes.byref(lat), 0.1, p(16), None, 0, 17, p(32), p(48), 1e-8, 10, p(64), 1 << 20,
                       info, None) == h.INVALID_ARG
    # reduced inner precision needs its links
    assert lib.hisq_cg(None, ctypes.byref(lat), 0.1, p(16), None, 1, 1, p(32), p(48), 1e-8, 10, p(64), 1 << 20,
                       info, None) == h.INVALID_ARG
    # multi-shift: m^2 + shift <= 0, aliasing solutions
    sh = (ctypes.c_double * 2)(-0.02, 0.1)
    tl = (ctypes.c_double * 2)(1e-8, 1e-8)
    xs = (ctypes.c_void_p * 2)(80, 96)
    assert lib.hisq_multishift_cg(None, ctypes.byref(lat), 0.1, p(16), None, 0, 2, sh, p(32), xs, tl, 10, p(64),
                                  1 << 20, info, None) == h.INVALID_ARG
    sh = (ctypes.c_double * 2)(0.0, 0.1)
    xs = (ctypes.c_void_p * 2)(80, 80)
    assert lib.hisq_multishift_cg(None, ctypes.byref(lat), 0.1, p(16), None, 0, 2, sh, p(32), xs, tl, 10, p(64),
                                  1 << 20, info, None) == h.INVALID_ARG


def test_workspace_queries(lib):
    from paper_2306_01098_amd import hisq as h
    lat = h.lattice((8, 8, 8, 8), -1)
    a = h.hisq_cg_workspace_bytes(lat, "fp64", 1, 0)
    b = h.hisq_cg_workspace_bytes(lat, "fp32", 16, 0)
    c = h.hisq_cg_workspace_bytes(lat, "fp32", 1, 14)
    assert 0 < a < b and a < c
    assert h.hisq_cg_workspace_bytes(lat, "fp64", 1, 33) == 0
    assert h.hisq_ptc_workspace_bytes(lat) > 2 * 8 * 4096 * 24   # two 8-channel activations
    assert h.hisq_fcg_workspace_bytes(lat) > h.hisq_ptc_workspace_bytes(lat)
    probs = (h.hisq_problem * 2)()
    probs[0].lat = h.lattice((8, 8, 8, 8), -1)
    probs[1].lat = h.lattice((4, 4, 4, 6), -1)
    assert lib.hisq_cg_batch_workspace_bytes(2, probs, 1) > 0
    assert lib.hisq_cg_batch_workspace_bytes(2, probs, 4) == 0     # no reconstruct-12 in the batch
    probs[1].lat = h.lattice((4, 4, 4, 5), -1)
    assert lib.hisq_cg_batch_workspace_bytes(2, probs, 1) == 0


def test_batch_and_ptc_argument_checks(lib):
    from paper_2306_01098_amd import hisq as h
    p = ctypes.c_void_p
    probs = (h.hisq_problem * 1)()
    probs[0].lat = h.lattice((4, 4, 4, 4), -1)
    probs[0].mass = 0.1
    probs[0].tol = 1e-8
    info = (h.hisq_solve_info * 1)()
    # NULL links / b / x
    assert lib.hisq_cg_batch(None, 1, probs, 0, 10, p(16), 1 << 20, info, None, None) == h.INVALID_ARG
    assert lib.hisq_cg_batch(None, 0, probs, 0, 10, p(16), 1 << 20, info, None, None) == h.INVALID_ARG
    lat = h.lattice((4, 4, 4, 4), -1)
    assert lib.hisq_ptc_forward(None, ctypes.byref(lat), None, p(16), p(32), p(48), p(64), 1 << 20,
                                None) == h.INVALID_ARG
    assert lib.hisq_ptc_adam_step(None, p(16), p(32), p(48), p(64), p(80), 0, 1e-3, 0.9, 0.999, 1e-8,
                                  None) == h.INVALID_ARG
    assert lib.hisq_fcg(None, ctypes.byref(lat), 0.1, p(16), p(24), p(32), p(40), p(40), 1e-8, 10, p(64),
                        1 << 20, None, None) == h.INVALID_ARG


def test_stream_copy_argument_checks(lib):
    from paper_2306_01098_amd import hisq as h
    p = ctypes.c_void_p
    # zero bytes, not a multiple of 16, misaligned, overlapping, NULL
    assert lib.hisq_stream_copy(None, p(4096), p(1 << 20), 0, None) == h.INVALID_ARG
    assert lib.hisq_stream_copy(None, p(4096), p(1 << 20), 24, None) == h.INVALID_ARG
    assert lib.hisq_stream_copy(None, p(4104), p(1 << 20), 32, None) == h.INVALID_ARG
    assert lib.hisq_stream_copy(None, p(4096), p(4096 + 16), 64, None) == h.INVALID_ARG
    assert b"overlap" in lib.hisq_last_error()
    assert lib.hisq_stream_copy(None, None, p(1 << 20), 64, None) == h.INVALID_ARG


def test_stream_read_argument_checks(lib):
    from paper_2306_01098_amd import hisq as h
    p = ctypes.c_void_p
    assert lib.hisq_stream_read_sink_words(16) == 1
    assert lib.hisq_stream_read_sink_words(16 * 1024) == 1
    assert lib.hisq_stream_read_sink_words(16 * 1025) == 2
    assert lib.hisq_stream_read_sink_words(24) == 0
    # zero bytes, not a multiple of 16, misaligned src or sink, overlap, NULL
    assert lib.hisq_stream_read(None, p(4096), 0, p(1 << 20), None) == h.INVALID_ARG
    assert lib.hisq_stream_read(None, p(4096), 24, p(1 << 20), None) == h.INVALID_ARG
    assert lib.hisq_stream_read(None, p(4104), 32, p(1 << 20), None) == h.INVALID_ARG
    assert lib.hisq_stream_read(None, p(4096), 32, p((1 << 20) + 2), None) == h.INVALID_ARG
    assert lib.hisq_stream_read(None, p(4096), 64, p(4096 + 16), None) == h.INVALID_ARG
    assert b"overlap" in lib.hisq_last_error()
    assert lib.hisq_stream_read(None, None, 64, p(1 << 20), None) == h.INVALID_ARG
    assert lib.hisq_stream_read(None, p(4096), 64, None, None) == h.INVALID_ARG


def test_condensate_argument_checks(lib):
    from paper_2306_01098_amd import hisq as h
    lat = ctypes.byref(h.lattice((4, 4, 4, 4), -1))
    p = ctypes.c_void_p
    out = ctypes.c_double()
    # nnoise 0, noise aliasing x, NULL pbp, mass 0
    assert lib.hisq_chiral_condensate(None, lat, 0.1, p(16), None, 0, 0, p(32), p(48), 1e-8, 10, p(64), 1 << 20,
                                      None, ctypes.byref(out), None, None, None) == h.INVALID_ARG
    assert lib.hisq_chiral_condensate(None, lat, 0.1, p(16), None, 0, 2, p(32), p(32), 1e-8, 10, p(64), 1 << 20,
                                      None, ctypes.byref(out), None, None, None) == h.INVALID_ARG
    assert lib.hisq_chiral_condensate(None, lat, 0.1, p(16), None, 0, 2, p(32), p(48), 1e-8, 10, p(64), 1 << 20,
                                      None, None, None, None, None) == h.INVALID_ARG
    assert lib.hisq_chiral_condensate(None, lat, 0.0, p(16), None, 0, 2, p(32), p(48), 1e-8, 10, p(64), 1 << 20,
                                      None, ctypes.byref(out), None, None, None) == h.INVALID_ARG


def test_smear_argument_checks(lib):
    from paper_2306_01098_amd import hisq as h
    lat = ctypes.byref(h.lattice((4, 4, 4, 4), -1))
    p = ctypes.c_void_p
    n = h.hisq_smear_workspace_bytes(h.lattice((4, 4, 4, 4), -1))
    assert n == 256 * 44 * 144
    assert lib.hisq_smear_links(None, lat, p(16), 0.0, p(16), p(48), p(64), n, None) == h.INVALID_ARG
    assert lib.hisq_smear_links(None, lat, p(16), 0.0, p(32), p(48), p(64), n - 1, None) == h.WORKSPACE
    assert lib.hisq_smear_links(None, lat, None, 0.0, p(32), p(48), p(64), n, None) == h.INVALID_ARG


def test_largest_volume_is_enforced(lib):
    from paper_2306_01098_amd import hisq as h
    ok = h.lattice((1024, 1024, 256, 4), -1)          # 2^30 sites: the limit
    big = h.lattice((1024, 1024, 512, 4), -1)         # 2^31 sites
    assert h.hisq_field_bytes(ok, "fp64", 1) == (1 << 29) * 48
    assert h.hisq_links_bytes(big, "fp64") == 0
    assert h.hisq_field_bytes(big, "fp32", 1) == 0
