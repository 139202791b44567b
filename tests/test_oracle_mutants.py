"""Plant plausible mistakes in a copy of the oracle's C source and check the pins catch each one.

The mutants are compiled into a temporary directory on the CPU; the real
oracle is never modified.  A mutant counts as caught when its results differ
from the brute-force path minimum, the hand-worked examples or the closed
forms used in test_oracle_pins.py.
"""
import ctypes
import itertools
import os
import subprocess

import numpy as np
import pytest

from oracle.brute import brute_dtw

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "dtw_oracle.c")

MUTANTS = {
    "drop_diagonal": ("double best = prev[j - 1];", "double best = INFINITY;"),
    "drop_up": ("if (prev[j] < best) best = prev[j];", ""),
    "drop_left": ("if (cur[j - 1] < best) best = cur[j - 1];\n            double d = x[i - 1] - y[j - 1];\n            cur[j]",
                  "double d = x[i - 1] - y[j - 1];\n            cur[j]"),
    "absolute_cost": ("cur[j] = d * d + best;", "cur[j] = fabs(d) + best;"),
    "shifted_x_index": ("double d = x[i - 1] - y[j - 1];\n            cur[j]", "double d = x[i - 1] - y[j > 1 ? j - 2 : 0];\n            cur[j]"),
    "window_ignores_length_gap": ("return (int64_t)w > d ? (int64_t)w : d;", "return (int64_t)w;"),
    "window_strict": ("if (off > b) {\n                cur[j]", "if (off >= b) {\n                cur[j]"),
    "zero_border": ("cur[0] = INFINITY;\n        for (int32_t j = 1; j <= m; ++j) {\n            int64_t off",
                    "cur[0] = 0.0;\n        for (int32_t j = 1; j <= m; ++j) {\n            int64_t off"),
    "max_instead_of_min": ("if (prev[j] < best) best = prev[j];", "if (prev[j] > best) best = prev[j];"),
}


def _build_mutant(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) >= 1, name
    text = text.replace(old, new, 1)
    src = tmp_path / (name + ".c")
    src.write_text(text)
    so = tmp_path / (name + ".so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                    "-o", str(so), str(src), "-lm"], check=True, capture_output=True)
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_dtw_pair.argtypes = [dp, ctypes.c_int32, dp, ctypes.c_int32, ctypes.c_int32, dp]
    lib.oracle_dtw_pair.restype = ctypes.c_double

    def dtw(x, y, w=-1):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        work = np.empty(2 * (len(y) + 1))
        return lib.oracle_dtw_pair(x.ctypes.data_as(dp), len(x), y.ctypes.data_as(dp), len(y), w,
                                   work.ctypes.data_as(dp))
    return dtw


def _pins_pass(dtw) -> bool:
    rng = np.random.default_rng(99)
    for w in (-1, 0, 1):
        for n, m in itertools.product(range(1, 5), range(1, 5)):
            x = rng.integers(-3, 4, size=n).astype(float)
            y = rng.integers(-3, 4, size=m).astype(float)
            best, _ = brute_dtw(x, y, w)
            if dtw(x, y, w) != float(best):
                return False
    # closed forms
    x = rng.standard_normal(12)
    if dtw(x, np.repeat(x, 2)) != 0.0:
        return False
    if dtw([1.5] * 5, [-0.5] * 9, 0) != 9 * 4.0:
        return False
    return True


def test_real_oracle_passes_the_same_checks(tmp_path):
    dtw = _build_mutant(tmp_path, "identity", "#include <math.h>", "#include <math.h>")
    assert _pins_pass(dtw)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    dtw = _build_mutant(tmp_path, name, old, new)
    assert not _pins_pass(dtw), "planted mistake %s was not detected" % name
