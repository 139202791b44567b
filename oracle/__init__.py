"""FP64 CPU oracle for the all-pairs DTW distance matrix.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the GPU
library (``paper_2307_04904_amd``) and never imports it.

The arithmetic lives in ``dtw_oracle.c`` (plain C, IEEE double, no fast-math);
this module compiles it with gcc on first use and wraps it with ctypes.
Definitions follow the paper's "Mathematical background" section: Eq. (c) for
the cell recurrence, the final cost c(n,m), and the symmetric distance matrix
D whose entries are the pairwise costs.  ``brute.py`` holds an independent
path-enumeration definition used to pin this module.

Window reading (paper, Introduction): cell (i,j) is admissible iff
|i-j| <= max(w, |n-m|); w < 0 means no window.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dtw_oracle.c")
_BUILD_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD_DIR, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile dtw_oracle.c into oracle/_build/liboracle.so with gcc."""
    os.makedirs(_BUILD_DIR, exist_ok=True)
    stale = (not os.path.exists(_LIB_PATH)) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC))
    if force or stale:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_band_cells.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_band_cells.restype = ctypes.c_int64
    lib.oracle_dtw_pair.argtypes = [dp, ctypes.c_int32, dp, ctypes.c_int32, ctypes.c_int32, dp]
    lib.oracle_dtw_pair.restype = ctypes.c_double
    lib.oracle_dtw_full.argtypes = [dp, ctypes.c_int32, dp, ctypes.c_int32, ctypes.c_int32, dp]
    lib.oracle_dtw_full.restype = ctypes.c_double
    lib.oracle_dtw_pairs.argtypes = [dp, i64p, i32p, ctypes.c_int32, i32p, i32p, i32p,
                                     ctypes.c_int64, dp, ctypes.c_int32]
    lib.oracle_dtw_pairs.restype = ctypes.c_int32
    lib.oracle_host_threads.argtypes = []
    lib.oracle_host_threads.restype = ctypes.c_int32
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_f64(v) -> np.ndarray:
    """Exact upcast of the stored values (f32/f16/bf16-as-f32/f64) to double."""
    return np.ascontiguousarray(np.asarray(v), dtype=np.float64)


def host_threads() -> int:
    return int(_load().oracle_host_threads())


def band_cells(n: int, m: int, window: int) -> int:
    """Number of admissible cells of an n x m problem under the window rule."""
    return int(_load().oracle_band_cells(int(n), int(m), int(window)))


def dtw(x, y, window: int = -1) -> float:
    """DTW cost c(n,m) of one pair, Eq. (c), two-row scheme, FP64."""
    x = _as_f64(x)
    y = _as_f64(y)
    work = np.empty(2 * (len(y) + 1), dtype=np.float64)
    return float(_load().oracle_dtw_pair(_dptr(x), len(x), _dptr(y), len(y), int(window), _dptr(work)))


def dtw_matrix(x, y, window: int = -1) -> np.ndarray:
    """The whole (n+1) x (m+1) cumulative-cost matrix of Eq. (c), 1-based borders included."""
    x = _as_f64(x)
    y = _as_f64(y)
    C = np.empty((len(x) + 1, len(y) + 1), dtype=np.float64)
    _load().oracle_dtw_full(_dptr(x), len(x), _dptr(y), len(y), int(window), _dptr(C))
    return C


def condensed_index(i: int, j: int, N: int) -> int:
    """Row-major index of pair (i, j), i < j, in the condensed upper triangle of D."""
    if i > j:
        i, j = j, i
    return i * N - i * (i + 1) // 2 + (j - i - 1)


def all_pairs_list(N: int):
    """(i, j) for every i < j in condensed order."""
    iu, ju = np.triu_indices(N, k=1)
    return iu.astype(np.int32), ju.astype(np.int32)


def dtw_pairs(values, offsets, lengths, pi, pj, window, threads: int = 0):
    """DTW of an explicit pair list over a ragged concatenated buffer.

    values: 1-D stored series values (any float dtype, upcast exactly);
    offsets/lengths: per-series start and length; pi/pj: pair endpoints;
    window: scalar or per-pair int.  Returns (float64 array, threads used).
    """
    lib = _load()
    v = _as_f64(values)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    ln = np.ascontiguousarray(lengths, dtype=np.int32)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    P = len(pi)
    win = np.ascontiguousarray(np.broadcast_to(np.asarray(window, dtype=np.int32), (P,)))
    out = np.empty(P, dtype=np.float64)
    if P == 0:
        return out, 0
    used = lib.oracle_dtw_pairs(
        _dptr(v), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        ln.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(ln),
        pi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        pj.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        win.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), P, _dptr(out), int(threads))
    if used < 0:
        raise MemoryError("oracle_dtw_pairs: allocation failed")
    return out, int(used)


def pairwise_condensed(values, offsets, lengths, window, threads: int = 0):
    """Condensed upper triangle of D (paper, Fig. "c_to_d"): all i < j, FP64."""
    N = len(lengths)
    pi, pj = all_pairs_list(N)
    out, _ = dtw_pairs(values, offsets, lengths, pi, pj, window, threads)
    return out
