"""Mutation check of the oracle's pins (CPU only).

Each mutant is a copy of oracle/oracle.c with one plausible slip planted (a
wrong sign, a dropped term, a transposed index, an off-by-one bound, a wrong
output size).  The copy is compiled into a temporary library and the pins of
test_oracle_pins.py are run against it; every mutant must make at least one
pin fail.  The real oracle is never modified.
"""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "pad_sign": ("i * stride - pad + ir", "i * stride + pad + ir"),
    "col_pad_dropped": ("j * stride - pad + is", "j * stride + is"),
    "weight_rs_transposed": ("* r + ir) * s + is]", "* r + is) * s + ir]"),
    "row_bound_off_by_one": ("yy < 0 || yy >= h || xx < 0 || xx >= w)\n                                    continue;",
                             "yy < 0 || yy > h || xx < 0 || xx >= w)\n                                    continue;"),
    "last_tap_dropped": ("for (int is = 0; is < s; ++is) {", "for (int is = 0; is < s - 1; ++is) {"),
    "input_channel_index": ("x[((size_t)(in * c + ic) * h + yy) * w + xx];\n", "x[((size_t)(in * c) * h + yy) * w + xx];\n"),
    "bias_sign": ("y[((size_t)in * k + ik) * hw + p] += b[ik];", "y[((size_t)in * k + ik) * hw + p] -= b[ik];"),
    "bn_eps_outside_sqrt": ("sqrt(var[ik] + eps)", "(sqrt(var[ik]) + eps)"),
    "bn_mean_sign": ("(*v - mean[ik])", "(*v + mean[ik])"),
    "bn_gamma_beta_swapped": ("gamma[ik] * (*v - mean[ik]) / sd + beta[ik]", "beta[ik] * (*v - mean[ik]) / sd + gamma[ik]"),
    "leaky_slope_sign": ("y[i] = slope * y[i];", "y[i] = -slope * y[i];"),
    "leaky_keeps_negatives": ("if (!(y[i] > 0.0))", "if (y[i] > 1e300)"),
    "pool_offset": ("const int off = (size - 1) / 2;", "const int off = size / 2;"),
    "pool_no_pad_size": ("const int ho = (h - 1) / stride + 1;", "const int ho = (h - size) / stride + 1;"),
    "pool_min": ("if (t > m)", "if (t < m || m == -INFINITY)"),
    "pool_window_short": ("for (int v = 0; v < size; ++v)", "for (int v = 0; v < size - 1; ++v)"),
    "shortcut_sign": ("y[i] += x[i];", "y[i] -= x[i];"),
}

PINS = [getattr(pins, n) for n in dir(pins) if n.startswith("test_")]


def _run_pins():
    failures = []
    for f in PINS:
        marks = getattr(f, "pytestmark", [])
        cases = [()]
        for m in marks:
            if m.name == "parametrize":
                cases = [tuple(c) for c in m.args[1]]
        for args in cases:
            try:
                f(*args)
            except (AssertionError, ValueError, IndexError) as e:  # a pin caught it
                failures.append((f.__name__, type(e).__name__))
                break
    return failures


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found: %s" % name
    mutated = src.replace(old, new, 1)
    cfile = tmp_path / "mut.c"
    cfile.write_text(mutated)
    lib = str(tmp_path / ("libmut_%s.so" % name))
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", lib, str(cfile), "-lm"])
    with oracle.use_library(lib):
        caught = _run_pins()
    assert caught, "mutant %s survived every pin" % name


def test_unmutated_passes_all_pins():
    assert _run_pins() == []
