"""Brute-force DTW by enumerating every warping path (tiny inputs only).

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is the plain definition that the dynamic programme of Eq. (c) solves,
written without any recursion on partial costs: a warping path is a sequence
of cells that starts at the first pair of points and ends at the last pair
(endpoints matched), never moves backwards in either series (monotonicity),
and advances by at most one point in each series per step, so that no point
is skipped (continuity) -- the three constraints listed in the paper's
"Mathematical background" section.  The cost of a path is the sum of the local
costs (x_i - y_j)^2 over its cells, and DTW is the minimum over all admissible
paths.  With a window w >= 0 every cell on the path must satisfy
|i - j| <= max(w, |n - m|).

Arithmetic is exact: every float converts exactly to a Fraction, so the
returned minimum is the true real-number value for the stored inputs.
"""
from __future__ import annotations

from fractions import Fraction

STEPS = ((1, 0), (0, 1), (1, 1))


def _admissible(i: int, j: int, band) -> bool:
    return band is None or abs(i - j) <= band


def enumerate_paths(n: int, m: int, window: int = -1):
    """Yield every admissible warping path as a tuple of 0-based (i, j) cells."""
    band = None if window < 0 else max(window, abs(n - m))
    if n <= 0 or m <= 0:
        return
    stack = [((0, 0),)]
    while stack:
        path = stack.pop()
        i, j = path[-1]
        if (i, j) == (n - 1, m - 1):
            yield path
            continue
        for di, dj in STEPS:
            a, b = i + di, j + dj
            if a < n and b < m and _admissible(a, b, band):
                stack.append(path + ((a, b),))


def brute_dtw(x, y, window: int = -1):
    """Return (exact minimum path cost as Fraction, number of admissible paths)."""
    xs = [Fraction(float(v)) for v in x]
    ys = [Fraction(float(v)) for v in y]
    best = None
    count = 0
    for path in enumerate_paths(len(xs), len(ys), window):
        count += 1
        cost = sum(((xs[i] - ys[j]) ** 2 for i, j in path), Fraction(0))
        if best is None or cost < best:
            best = cost
    return best, count
