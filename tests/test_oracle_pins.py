"""Pins for the FP64 oracle: results it must reproduce that do not come from itself.

Each test compares the oracle with something fixed independently of its code:
the path-enumeration definition (exact rationals), the Delannoy path count,
a library shortest-path routine on the DTW grid graph, closed forms, exact
invariants and hand-worked examples.  Together they catch a dropped
predecessor, a swapped index, a wrong border, a wrong window rule or a
missing square (see test_oracle_mutants.py, which plants such mistakes).
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

import oracle
from oracle.brute import brute_dtw

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.txt")


def delannoy(a: int, b: int) -> int:
    """Number of lattice paths with steps E, N, NE from (0,0) to (a,b) (closed form)."""
    return sum(math.comb(a, k) * math.comb(b, k) * 2 ** k for k in range(min(a, b) + 1))


# ---------------------------------------------------------------- definitions

def test_hand_examples():
    n_cases = 0
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            xs, ys, w, expected, _why = [p.strip() for p in line.split(";", 4)]
            x = [float(t) for t in xs.split()]
            y = [float(t) for t in ys.split()]
            assert oracle.dtw(x, y, int(w)) == float(expected), line
            best, _ = brute_dtw(x, y, int(w))
            assert best == Fraction(expected), line
            n_cases += 1
    assert n_cases >= 8


@pytest.mark.parametrize("window", [-1, 0, 1, 2])
def test_brute_force_small_integer(window):
    """Every n, m <= 5 with small integer data: the DP equals the minimum over all paths, exactly."""
    rng = np.random.default_rng(1000 + window)
    for n, m in itertools.product(range(1, 6), range(1, 6)):
        for _ in range(2):
            x = rng.integers(-3, 4, size=n).astype(float)
            y = rng.integers(-3, 4, size=m).astype(float)
            best, count = brute_dtw(x, y, window)
            assert count >= 1
            assert oracle.dtw(x, y, window) == float(best), (n, m, window, x, y)


def test_brute_force_six_by_six_and_float():
    rng = np.random.default_rng(7)
    x = rng.integers(-3, 4, size=6).astype(float)
    y = rng.integers(-3, 4, size=6).astype(float)
    best, count = brute_dtw(x, y, -1)
    assert count == 1683
    assert oracle.dtw(x, y) == float(best)
    # non-integer data: FP64 result within the rounding bound of the exact rational minimum
    for n, m in [(4, 5), (5, 3), (6, 4)]:
        xf = rng.standard_normal(n)
        yf = rng.standard_normal(m)
        best, _ = brute_dtw(xf, yf, -1)
        got = oracle.dtw(xf, yf)
        assert abs(Fraction(got) - best) <= Fraction(2 * (n + m)) * Fraction(2) ** -52 * best


def test_path_count_is_delannoy():
    for n, m in itertools.product(range(1, 6), range(1, 6)):
        _, count = brute_dtw([0.0] * n, [0.0] * m, -1)
        assert count == delannoy(n - 1, m - 1)
    assert [delannoy(k, k) for k in range(6)] == [1, 3, 13, 63, 321, 1683]


def _grid_shortest_path(x, y, window):
    """DTW as a node-weighted shortest path on the grid DAG, solved by scipy's Dijkstra."""
    n, m = len(x), len(y)
    band = None if window < 0 else max(window, abs(n - m))
    node = lambda i, j: 1 + i * m + j  # node 0 is a source
    rows, cols, vals = [], [], []

    def ok(i, j):
        return band is None or abs(i - j) <= band

    cost = lambda i, j: (x[i] - y[j]) ** 2 + 1e-300  # keep explicit zeros as edges
    rows.append(0); cols.append(node(0, 0)); vals.append(cost(0, 0))
    for i in range(n):
        for j in range(m):
            if not ok(i, j):
                continue
            for di, dj in ((1, 0), (0, 1), (1, 1)):
                a, b = i + di, j + dj
                if a < n and b < m and ok(a, b):
                    rows.append(node(i, j)); cols.append(node(a, b)); vals.append(cost(a, b))
    g = sp.csr_matrix((vals, (rows, cols)), shape=(1 + n * m, 1 + n * m))
    dist = dijkstra(g, directed=True, indices=0)
    return dist[node(n - 1, m - 1)]


@pytest.mark.parametrize("n,m,window", [(30, 45, -1), (40, 40, 3), (25, 37, 5), (37, 25, 0), (33, 33, 0), (50, 20, 40)])
def test_matches_library_shortest_path(n, m, window):
    rng = np.random.default_rng(n * 100 + m)
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    ref = _grid_shortest_path(x, y, window)
    got = oracle.dtw(x, y, window)
    assert got == pytest.approx(ref, rel=1e-12, abs=1e-250)


# ---------------------------------------------------------------- closed forms

def test_window_zero_is_squared_euclidean():
    rng = np.random.default_rng(3)
    for L in [1, 2, 17, 300]:
        x = rng.standard_normal(L)
        y = rng.standard_normal(L)
        ref = float(np.sum((x - y) ** 2))
        assert oracle.dtw(x, y, 0) == pytest.approx(ref, rel=1e-13)
    xi = rng.integers(-5, 6, size=64).astype(float)
    yi = rng.integers(-5, 6, size=64).astype(float)
    assert oracle.dtw(xi, yi, 0) == float(np.sum((xi - yi) ** 2))


def test_singleton_series():
    rng = np.random.default_rng(4)
    x = rng.integers(-5, 6, size=23).astype(float)
    y1 = np.array([2.0])
    expected = float(np.sum((x - 2.0) ** 2))
    for w in [-1, 0, 3]:
        assert oracle.dtw(x, y1, w) == expected
        assert oracle.dtw(y1, x, w) == expected


def test_constant_series():
    for n, m in [(5, 9), (9, 5), (7, 7), (1, 12)]:
        for w in [-1, 0, 2]:
            assert oracle.dtw([1.5] * n, [-0.5] * m, w) == max(n, m) * 4.0


def test_identity_is_exact_zero():
    rng = np.random.default_rng(5)
    for L in [1, 8, 200]:
        x = rng.standard_normal(L)
        for w in [-1, 0, 5]:
            assert oracle.dtw(x, x, w) == 0.0


def test_upsampled_copy_is_zero():
    rng = np.random.default_rng(6)
    x = rng.standard_normal(31)
    assert oracle.dtw(x, np.repeat(x, 2), -1) == 0.0
    assert oracle.dtw(np.repeat(x, 3), x, -1) == 0.0


# ---------------------------------------------------------------- invariants

def test_symmetry_bitwise():
    rng = np.random.default_rng(8)
    for n, m, w in [(40, 55, -1), (64, 64, 6), (17, 90, 0)]:
        x = rng.standard_normal(n)
        y = rng.standard_normal(m)
        assert oracle.dtw(x, y, w) == oracle.dtw(y, x, w)


def test_window_monotone_bitwise():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(80)
    y = rng.standard_normal(80)
    vals = [oracle.dtw(x, y, w) for w in range(0, 80)] + [oracle.dtw(x, y, -1)]
    assert all(b <= a for a, b in zip(vals, vals[1:]))
    assert vals[79] == vals[80]  # window >= n-1 is the same as no window


def test_power_of_two_scaling_bitwise():
    rng = np.random.default_rng(10)
    x = rng.standard_normal(50)
    y = rng.standard_normal(61)
    base = oracle.dtw(x, y, 7)
    for k in [-3, 1, 4]:
        assert oracle.dtw(x * 2.0 ** k, y * 2.0 ** k, 7) == base * 4.0 ** k


def test_shift_and_reversal():
    rng = np.random.default_rng(11)
    x = rng.standard_normal(70)
    y = rng.standard_normal(70)
    base = oracle.dtw(x, y, 9)
    assert oracle.dtw(x + 3.25, y + 3.25, 9) == pytest.approx(base, rel=1e-12)
    assert oracle.dtw(x[::-1], y[::-1], 9) == pytest.approx(base, rel=1e-12)
    z = rng.standard_normal(45)
    assert oracle.dtw(x[::-1], z[::-1]) == pytest.approx(oracle.dtw(x, z), rel=1e-12)


def test_bounds():
    rng = np.random.default_rng(12)
    for _ in range(20):
        n, m = rng.integers(2, 60, size=2)
        x = rng.standard_normal(n)
        y = rng.standard_normal(m)
        d = oracle.dtw(x, y)
        assert d >= (x[0] - y[0]) ** 2 + (x[-1] - y[-1]) ** 2 - 1e-12
        if n == m:
            assert d <= float(np.sum((x - y) ** 2)) + 1e-12


def test_rolling_equals_full_matrix_bitwise():
    rng = np.random.default_rng(13)
    for n, m, w in [(30, 41, -1), (41, 30, 4), (25, 25, 0), (1, 9, -1)]:
        x = rng.standard_normal(n)
        y = rng.standard_normal(m)
        C = oracle.dtw_matrix(x, y, w)
        assert C[n, m] == oracle.dtw(x, y, w)
        assert C[0, 0] == 0.0 and np.all(np.isinf(C[0, 1:])) and np.all(np.isinf(C[1:, 0]))


def test_band_cell_count():
    for n, m, w in [(512, 512, 51), (256, 256, 25), (64, 64, -1), (4096, 4096, -1), (30, 70, 5), (70, 30, 0), (9, 9, 0)]:
        i = np.arange(n)[:, None]
        j = np.arange(m)[None, :]
        band = np.inf if w < 0 else max(w, abs(n - m))
        assert oracle.band_cells(n, m, w) == int(np.count_nonzero(np.abs(i - j) <= band))
    assert oracle.band_cells(512, 512, 51) == 50084
    assert oracle.band_cells(256, 256, 25) == 12406


def test_pairs_driver_matches_single_calls():
    rng = np.random.default_rng(14)
    lens = rng.integers(1, 40, size=9)
    series = [rng.standard_normal(L) for L in lens]
    values = np.concatenate(series)
    offsets = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    D = oracle.pairwise_condensed(values, offsets, lens, 3, threads=3)
    k = 0
    for i in range(9):
        for j in range(i + 1, 9):
            assert oracle.condensed_index(i, j, 9) == k
            assert D[k] == oracle.dtw(series[i], series[j], 3)
            k += 1
    assert k == len(D)
