"""FP64 CPU oracle for the optimal warping path of one pair.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It shares no code with the GPU
library and never imports it.

The paper (Mathematical background, Fig. 1) shows the cumulative-cost matrix
C of Eq. (c) for one pair and the warping path through it: the sequence of
matched cells from (1,1) to (n,m) whose local costs sum to c(n,m).  The path
is recovered by walking back from (n,m): at each cell, move to the
predecessor (diagonal (i-1,j-1), up (i-1,j) or left (i,j-1)) holding the
smallest cumulative cost.  Several optimal paths can exist; this module
breaks ties in the order diagonal, up, left.  Cells are 0-based here:
(0,0) .. (n-1,m-1).
"""
from __future__ import annotations

import numpy as np

import oracle


def backtrack(C) -> list:
    """Optimal path through a cumulative-cost matrix with 1-based borders
    (shape (n+1, m+1), C[0,0] = 0, other border cells +inf), as 0-based cells."""
    C = np.asarray(C, dtype=np.float64)
    i, j = C.shape[0] - 1, C.shape[1] - 1
    path = [(i - 1, j - 1)]
    while (i, j) != (1, 1):
        cands = ((C[i - 1, j - 1], i - 1, j - 1), (C[i - 1, j], i - 1, j), (C[i, j - 1], i, j - 1))
        best = min(c[0] for c in cands)
        _, i, j = next(c for c in cands if c[0] == best)  # first of diagonal, up, left
        path.append((i - 1, j - 1))
    return path[::-1]


def path_cost(x, y, path) -> float:
    """Sum of the local costs (x_i - y_j)^2 over the cells of a path, FP64."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(sum((x[i] - y[j]) ** 2 for i, j in path))


def is_valid_path(path, n: int, m: int, window: int = -1) -> bool:
    """Starts at (0,0), ends at (n-1,m-1), moves by (1,0), (0,1) or (1,1), stays in the window."""
    band = None if window < 0 else max(window, abs(n - m))
    if not path or tuple(path[0]) != (0, 0) or tuple(path[-1]) != (n - 1, m - 1):
        return False
    for (a, b), (c, d) in zip(path, path[1:]):
        if (c - a, d - b) not in ((1, 0), (0, 1), (1, 1)):
            return False
    return band is None or all(abs(i - j) <= band for i, j in path)


def warping_path(x, y, window: int = -1):
    """(path, cost): an optimal warping path of the pair and c(n, m)."""
    C = oracle.dtw_matrix(x, y, window)
    return backtrack(C), float(C[-1, -1])
