"""Mutation check of the oracle pins (CPU only).

Each mutation below plants one plausible mistake in a copy of the C oracle
(``oracle/hisq_oracle.c``): a wrong staggered phase, a wrong link site, a
missing dagger, a misplaced boundary sign, a flipped Naik sign, a transposed
link, a wrong hop length.  The copy is compiled with gcc into a temporary
directory and substituted for the oracle library inside the test only; the
pins of ``test_oracle_dslash.py`` (closed forms, anti-Hermiticity, gauge
covariance, translation, the dense matrix built from the definition) are then
run against it, and at least one of them must fail for every mutant.  The
unaltered source, built the same way, must pass them all.
"""
import os
import shutil
import subprocess

import pytest

from oracle import hisq as O

import test_oracle_dslash as P

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCE = os.path.join(ROOT, "oracle", "hisq_oracle.c")

# name -> (text in the oracle source, replacement); each text occurs once
MUTATIONS = {
    "eta_sign": ("return (s & 1) ? -1.0 : 1.0;", "return (s & 1) ? 1.0 : -1.0;"),
    "eta_range": ("for (int nu = 0; nu < mu; ++nu)", "for (int nu = 0; nu <= mu; ++nu)"),
    "backward_link_site": ("mul_adj_add(acc, -e * sg, &X[((long)mu * V + nb) * 9]",
                           "mul_adj_add(acc, -e * sg, &X[((long)mu * V + s) * 9]"),
    "missing_dagger": ("mul_adj_add(acc, -e * sg, &X[", "mul_add(acc, -e * sg, &X["),
    "bc_direction": ("if (mu == 3)\n            sign = (double)t_bc;",
                     "if (mu == 2)\n            sign = (double)t_bc;"),
    "bc_forward_only": ("if (mu == 3)\n            sign = (double)t_bc;",
                        "if (mu == 3 && k > 0)\n            sign = (double)t_bc;"),
    "naik_sign": ("mul_add(acc, e * sg, &W[", "mul_add(acc, -e * sg, &W["),
    "transposed_link": ("acc += U[3 * a + b] * psi[b];", "acc += U[3 * b + a] * psi[b];"),
    "naik_hop_length": ("sg = hop(c, dims, mu, -3, t_bc, d);", "sg = hop(c, dims, mu, -1, t_bc, d);"),
}

# the pins, each a call of a test of test_oracle_dslash.py with fixed arguments
PINS = {
    "plane_wave_periodic": lambda: P.test_free_field_plane_wave_pointwise(+1, (0.7, -0.3)),
    "plane_wave_antiperiodic": lambda: P.test_free_field_plane_wave_pointwise(-1, (0.7, -0.3)),
    "plane_wave_naik_only": lambda: P.test_free_field_plane_wave_pointwise(-1, (0.0, 1.0)),
    "dense_blocks": lambda: P.test_dense_matches_oracle_and_blocks(-1),
    "anti_hermiticity": lambda: P.test_anti_hermiticity((4, 6, 8, 6), -1),
    "gauge_covariance": lambda: P.test_gauge_covariance(-1),
    "translation_t": lambda: P.test_translation_by_two_sites(3, -1),
    "translation_x": lambda: P.test_translation_by_two_sites(0, -1),
}


def build(src_text: str, out_dir: str) -> str:
    c = os.path.join(out_dir, "hisq_oracle.c")
    with open(c, "w") as fh:
        fh.write(src_text)
    so = os.path.join(out_dir, "liboracle_mut.so")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", so, c])
    return so


def failing_pins(so: str):
    failed = []
    with O.substituted_library(so):
        for name, pin in PINS.items():
            try:
                pin()
            except AssertionError:
                failed.append(name)
    return failed


@pytest.fixture(scope="module")
def source():
    with open(SOURCE) as fh:
        return fh.read()


def test_unaltered_oracle_passes_every_pin(source, tmp_path):
    assert shutil.which("gcc")
    assert failing_pins(build(source, str(tmp_path))) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutant_is_caught(source, tmp_path, name):
    old, new = MUTATIONS[name]
    assert source.count(old) == 1, name
    failed = failing_pins(build(source.replace(old, new), str(tmp_path)))
    assert failed, f"mutation {name} passed every pin"
    print(f"\n{name}: caught by {failed}")
