"""GPU warping path (dtw_path through the C ABI) against the FP64 path oracle.

Integer-valued series keep every cumulative cost exact in FP32, so the GPU
walk must reproduce the oracle's path cell for cell, ties included, and its
cost matrix exactly.  Real-valued series are compared by what is unique: the
GPU path is admissible, its FP64 cost is optimal within the FP32 rounding of
the sums, and its reported cost equals the PLAIN distance-matrix entry of the
pair bit for bit."""
import numpy as np
import pytest

import oracle
from oracle import path as opath

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    from paper_2307_04904_amd import binding
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return binding


def _int_series(seed, n, m, lo=-3, hi=4):
    rng = np.random.default_rng(seed)
    return (rng.integers(lo, hi, size=n).astype(np.float32), rng.integers(lo, hi, size=m).astype(np.float32))


def _real_series(seed, n, m):
    rng = np.random.default_rng(seed)
    # random walks, the shape of the paper's series
    return (np.cumsum(rng.standard_normal(n)).astype(np.float32),
            np.cumsum(rng.standard_normal(m)).astype(np.float32))


def _run(B, x, y, window, want_C=False):
    dx = torch.from_numpy(x).cuda()
    dy = torch.from_numpy(y).cuda()
    C = torch.full((len(x) * len(y),), -1.0, dtype=torch.float32, device="cuda") if want_C else None
    p, cost = B.warping_path(dx, dy, window, C_out=C)
    torch.cuda.synchronize()
    p = [tuple(map(int, r)) for r in p.cpu().numpy()]
    return p, cost, (C.cpu().numpy().reshape(len(x), len(y)) if want_C else None)


def _pairwise_entry(B, x, y, window):
    # the path's cost is a plain FP32 sum: compare with the plainly summed matrix entry
    series = torch.from_numpy(np.concatenate([x, y])).cuda()
    out = torch.empty(1, dtype=torch.float32, device="cuda")
    B.dtw_pairwise_ex(series, [len(x), len(y)], [0, len(x)], window, out, accum="plain")
    torch.cuda.synchronize()
    return float(out.cpu()[0])


# shapes cover every sweep shape (shorter series 1..64, ..512, 1024, 2048, 4096, 8192),
# both orientations (x shorter and x longer), ragged lane strips and one-point series
SHAPES = [(1, 1), (1, 7), (7, 1), (5, 5), (64, 64), (65, 129), (129, 65), (300, 517), (517, 300),
          (700, 1024), (1500, 1600), (3000, 2049), (4096, 4100), (5000, 4500)]


@pytest.mark.parametrize("n,m", SHAPES)
@pytest.mark.parametrize("window", [-1, 0, 7])
def test_integer_series_path_is_the_oracle_path(n, m, window):
    B = _gpu()
    print("dtw_path integer n=%d m=%d w=%d" % (n, m, window), flush=True)
    x, y = _int_series(n * 31 + m + window, n, m)
    want_C = n * m <= 2_000_000
    p, cost, C = _run(B, x, y, window, want_C)
    Cref = oracle.dtw_matrix(x, y, window)
    p_ref = opath.backtrack(Cref)
    assert cost == Cref[-1, -1]
    assert p == [tuple(c) for c in p_ref]
    if want_C:
        np.testing.assert_array_equal(C.astype(np.float64), Cref[1:, 1:])
        # without the matrix the sweep stores only the moves (2 bits a cell): the same walk
        p2, cost2, _ = _run(B, x, y, window)
        assert p2 == p and cost2 == cost


@pytest.mark.parametrize("n,m", [(1, 3), (40, 40), (64, 200), (333, 129), (1000, 1000), (2500, 2100)])
@pytest.mark.parametrize("window", [-1, 3, 50])
def test_real_series_path_is_optimal(n, m, window):
    B = _gpu()
    print("dtw_path real n=%d m=%d w=%d" % (n, m, window), flush=True)
    x, y = _real_series(1000 + n + 7 * m + window, n, m)
    p, cost, _ = _run(B, x, y, window)
    assert opath.is_valid_path(p, n, m, window)
    best = oracle.dtw(x, y, window)
    L = len(p)
    tol = (1e-5 if L <= 4096 else 1e-4) * max(best, 1e-30)
    assert abs(opath.path_cost(x, y, p) - best) <= tol
    assert abs(cost - best) <= tol
    assert cost == _pairwise_entry(B, x, y, window)


def test_cost_matrix_marks_inadmissible_cells():
    B = _gpu()
    x, y = _real_series(5, 90, 70)
    _, _, C = _run(B, x, y, 4, want_C=True)
    band = max(4, 20)
    i, j = np.indices(C.shape)
    assert np.all(np.isinf(C[np.abs(i - j) > band]))
    assert np.all(np.isfinite(C[np.abs(i - j) <= band]))
    Cref = oracle.dtw_matrix(x, y, 4)[1:, 1:]
    ok = np.isfinite(Cref)
    np.testing.assert_allclose(C[ok], Cref[ok], rtol=1e-5, atol=1e-6)


def test_equal_series_give_the_diagonal():
    B = _gpu()
    x, _ = _real_series(9, 2000, 1)
    p, cost, _ = _run(B, x, x.copy(), -1)
    assert cost == 0.0
    assert p == [(k, k) for k in range(2000)]


def test_all_ties_walk_diagonal_then_up():
    # every path costs 0: the walk back takes the diagonal while it can, then moves up
    B = _gpu()
    n, m = 300, 120
    p, cost, _ = _run(B, np.zeros(n, np.float32), np.zeros(m, np.float32), -1)
    assert cost == 0.0
    assert p == [(k, 0) for k in range(n - m + 1)] + [(n - m + k, k) for k in range(1, m)]


def test_longest_supported_shorter_series():
    # the shorter series at the 32768-point limit (widest sweep shape); the
    # full oracle matrix would not fit a test, so check what holds at any
    # size: an admissible path whose exact (integer) cost is the GPU cost and
    # the PLAIN distance-matrix entry of the pair
    B = _gpu()
    n, m = 32768, 33000
    print("dtw_path n=%d m=%d w=200" % (n, m), flush=True)
    x, y = _int_series(77, n, m, -2, 3)
    p, cost, _ = _run(B, x, y, 200)
    assert opath.is_valid_path(p, n, m, 200)
    assert opath.path_cost(x, y, p) == cost
    assert cost == _pairwise_entry(B, x, y, 200)
    assert cost == oracle.dtw(x, y, 200)


def test_repeated_calls_and_caller_stream():
    B = _gpu()
    x, y = _int_series(3, 500, 800)
    ref = opath.warping_path(x, y, 11)
    s = torch.cuda.Stream()
    dx, dy = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    buf = torch.empty(2 * (500 + 800 - 1), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    for _ in range(3):
        p, cost = B.warping_path(dx, dy, 11, path_out=buf, stream=s)
        assert [tuple(map(int, r)) for r in p.cpu().numpy()] == [tuple(c) for c in ref[0]]
        assert cost == ref[1]


def test_move_buffer_kept_between_calls_of_changing_size():
    # the moves-only form keeps its buffer between calls and grows it: calls
    # of increasing, then decreasing size, each checked against the oracle
    B = _gpu()
    for k, (n, m) in enumerate([(200, 300), (2600, 2500), (90, 1400), (3100, 3300), (64, 65)]):
        x, y = _int_series(500 + k, n, m)
        p, cost, _ = _run(B, x, y, 40)
        ref = opath.warping_path(x, y, 40)
        assert p == [tuple(c) for c in ref[0]], (n, m)
        assert cost == ref[1]
