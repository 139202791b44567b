"""Pins of the warping-path oracle (CPU): every path it returns is admissible
and optimal, checked against brute-force enumeration of all warping paths."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute, path


@pytest.mark.parametrize("n,m", [(1, 1), (1, 4), (4, 1), (2, 3), (3, 3), (4, 5), (5, 5), (6, 4)])
@pytest.mark.parametrize("window", [-1, 0, 1, 2])
def test_path_is_admissible_and_optimal(n, m, window):
    rng = np.random.default_rng(n * 10 + m + 100 * (window + 1))
    x = rng.integers(-3, 4, size=n).astype(np.float64)
    y = rng.integers(-3, 4, size=m).astype(np.float64)
    p, cost = path.warping_path(x, y, window)
    assert path.is_valid_path(p, n, m, window)
    best, _ = brute.brute_dtw(x, y, window)
    assert Fraction(path.path_cost(x, y, p)) == best == Fraction(cost)


def test_ties_prefer_diagonal_then_up_then_left():
    # all-equal series: every admissible path costs 0; the walk back takes the
    # diagonal while it can, then moves up
    p, cost = path.warping_path(np.zeros(5), np.zeros(3), -1)
    assert cost == 0.0
    assert p == [(0, 0), (1, 0), (2, 0), (3, 1), (4, 2)]
    # a left move only when the diagonal and up predecessors cost more
    p, _ = path.warping_path([0.0, 0.0], [0.0, 5.0, 0.0], -1)
    assert p == [(0, 0), (0, 1), (1, 2)]


def test_validity_checker_rejects_bad_paths():
    assert not path.is_valid_path([(0, 0), (2, 1)], 3, 2)
    assert not path.is_valid_path([(0, 0), (1, 1)], 3, 2)
    assert not path.is_valid_path([(0, 0), (1, 0), (2, 0), (2, 1), (2, 2)], 3, 3, window=1)
    assert path.is_valid_path([(0, 0), (1, 1), (2, 2)], 3, 3, window=0)


def test_known_example_from_the_hand_examples():
    # x = 1 2 3, y = 1 3: cost 1 along (1,1)(2,1)(3,2) (1-based)
    p, cost = path.warping_path([1.0, 2.0, 3.0], [1.0, 3.0])
    assert cost == 1.0 and p == [(0, 0), (1, 0), (2, 1)]
