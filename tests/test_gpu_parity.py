"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances, against the oracle run on the same stored values: relative
error <= 1e-5 for FP32 inputs and for Kahan-compensated FP32 sums on any
input; <= 1e-3 for BF16/FP16 inputs with plain FP32 sums; the FP64 mode must
equal the oracle rounded once to FP32.
A reference value of exactly 0 must come out exactly 0.
"""
import numpy as np
import pytest

import oracle
from paper_2307_04904_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL_TOL = 1e-5
REL_TOL_16BIT_PLAIN = 1e-3
REL_TOL_LONG_PLAIN = 1e-4  # plain FP32 sums along warping paths of more than 2048 cells


def plain_tol(ds):
    """Tolerance of plain FP32 sums for a dataset: each add along a path of k
    cells rounds once, so the relative error is about sqrt(k) * 2^-24 for
    random rounding (bounded by (k-1) * 2^-24); 1e-5 holds up to paths of
    2048 cells, longer paths get 1e-4 (the compensated modes keep 1e-5); data
    whose cheapest paths hug the band edge (many near-ties) reached 1.5e-5 at
    3,650-cell paths."""
    L = np.sort(np.asarray(ds.lengths, dtype=np.int64))
    longest_path = int(L[-1] + L[-2] - 1) if L.size > 1 else 0
    return REL_TOL if longest_path <= 2048 else REL_TOL_LONG_PLAIN


def _gpu():
    from paper_2307_04904_amd import binding
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return binding


def oracle_pairs(ds, pi, pj):
    vals = synth.stored_as_f64(ds)
    out, _ = oracle.dtw_pairs(vals, ds.offsets, ds.lengths, pi, pj, ds.window)
    return out


def condensed(pi, pj, N):
    pi = np.asarray(pi, dtype=np.int64)
    pj = np.asarray(pj, dtype=np.int64)
    return pi * N - pi * (pi + 1) // 2 + (pj - pi - 1)


def sample_pairs(N, k, seed):
    rng = np.random.default_rng(seed)
    i = rng.integers(0, N, size=4 * k)
    j = rng.integers(0, N, size=4 * k)
    keep = i != j
    a = np.minimum(i, j)[keep][:k]
    b = np.maximum(i, j)[keep][:k]
    # always include the first and last pairs
    a = np.concatenate([[0, N - 2], a]).astype(np.int32)
    b = np.concatenate([[1, N - 1], b]).astype(np.int32)
    return a, b


def assert_close(got, ref, tol=REL_TOL, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got)), what + ": non-finite output"
    zero = ref == 0.0
    assert np.all(got[zero] == 0.0), what + ": reference 0 not reproduced exactly"
    rel = np.abs(got[~zero] - ref[~zero]) / ref[~zero]
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= tol, "%s: max rel err %.3e > %.1e (mean %.3e)" % (what, worst, tol, float(rel.mean()))
    return worst


def run(ds, **kw):
    B = _gpu()
    out = B.pairwise(ds, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


# ---------------------------------------------------------------- small cases, every pair

@pytest.mark.parametrize("kernel", ["auto", "lane", "wave"])
def test_smallest_config_all_pairs(kernel):
    ds = synth.config1()
    got = run(ds, kernel=kernel)
    pi, pj = oracle.all_pairs_list(ds.N)
    assert_close(got, oracle_pairs(ds, pi, pj), what="20x64 full " + kernel)


@pytest.mark.parametrize("window", [-1, 0, 1, 5, 40])
def test_ragged_lengths_wavefront(window):
    # lengths 1..300 span strip heights 1..8, several ragged tails and both orientations
    ds = synth.small_random(seed=100 + max(window, 0), N=23, len_lo=1, len_hi=300, window=window)
    ds.lengths[0] = 1
    got = run(ds)
    pi, pj = oracle.all_pairs_list(ds.N)
    assert_close(got, oracle_pairs(ds, pi, pj), what="ragged w=%d" % window)


@pytest.mark.parametrize("window", [0, 3, 17, 36, 63, -1])
def test_equal_lengths_both_kernels(window):
    # N=150: every series has 74-75 partners -> one full and one ragged 64-lane item each
    ds = synth.small_random(seed=7, N=150, len_lo=37, len_hi=37, window=window)
    lane = run(ds, kernel="lane")
    wave = run(ds, kernel="wave")
    pi, pj = oracle.all_pairs_list(ds.N)
    ref = oracle_pairs(ds, pi, pj)
    assert_close(lane, ref, what="lane w=%d" % window)
    assert_close(wave, ref, what="wave w=%d" % window)
    # same per-cell arithmetic (sub, min of three, fused multiply-add) in both families
    assert np.array_equal(lane, wave)


@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 17])
def test_short_equal_lengths_lane_kernel(L):
    # lengths below and around the number of rows the lane kernel sweeps together
    ds0 = synth.small_random(seed=20 + L, N=70, len_lo=L, len_hi=L)
    pi, pj = oracle.all_pairs_list(ds0.N)
    for w in sorted({0, 1, L // 2, L - 1, -1}):
        ds = synth.pack([ds0.series(s).astype(np.float64) for s in range(ds0.N)], "short", w)
        lane = run(ds, kernel="lane")
        assert_close(lane, oracle_pairs(ds, pi, pj), what="lane L=%d w=%d" % (L, w))
        assert np.array_equal(lane, run(ds, kernel="wave"))


def test_long_strips_and_unequal_lengths():
    # pairs whose shorter series needs 12..64 rows per lane, window active on some
    rng = np.random.default_rng(5)
    lens = [700, 1500, 2900, 4096, 3100, 64, 1]
    series = [synth.random_walk(rng, L) for L in lens]
    for w in (-1, 150):
        ds = synth.pack(series, "long", w)
        got = run(ds)
        pi, pj = oracle.all_pairs_list(ds.N)
        assert_close(got, oracle_pairs(ds, pi, pj), what="long w=%d" % w)


@pytest.mark.parametrize("accum", ["plain", "kahan", "fp64"])
def test_series_longer_than_one_wavefront(accum):
    # shorter series of 4097..9000 points: strips spread over 2..8 wavefronts of a workgroup
    rng = np.random.default_rng(17)
    lens = [4097, 5000, 9000, 7000] if accum == "plain" else [4097, 5200, 3000]
    series = [synth.random_walk(rng, L) for L in lens]
    for w in (-1, 700):
        ds = synth.pack(series, "long%s" % accum, w)
        got = run(ds, accum=accum)
        pi, pj = oracle.all_pairs_list(ds.N)
        ref = oracle_pairs(ds, pi, pj)
        if accum == "fp64":
            assert np.array_equal(got, ref.astype(np.float32))
        else:
            # plain FP32 sums over paths of up to 16,000 cells drift past 1e-5 (each add rounds;
            # relative error bound (k-1)*2^-24); the compensated sums keep 1e-5
            assert_close(got, ref, tol=REL_TOL_LONG_PLAIN if accum == "plain" else REL_TOL,
                         what="long %s w=%d" % (accum, w))
        if accum == "plain":
            # windowed pairs go to the cyclic kernel by default; the multi-wavefront
            # strips (window events per lane, boundary rows through LDS) must agree bit for bit
            assert np.array_equal(run(ds, kernel="wave"), got), "long w=%d: strips differ" % w


@pytest.mark.parametrize("accum", ["kahan", "fp64"])
def test_precision_modes_ragged_windows(accum):
    ds = synth.small_random(seed=61, N=25, len_lo=1, len_hi=1100, window=37)
    got = run(ds, accum=accum)
    pi, pj = oracle.all_pairs_list(ds.N)
    ref = oracle_pairs(ds, pi, pj)
    if accum == "fp64":
        assert np.array_equal(got, ref.astype(np.float32))
    else:
        assert_close(got, ref, what="ragged %s" % accum)


def test_single_point_series_and_two_series():
    ds = synth.pack([np.array([0.5]), np.array([-1.0])], "tiny", 0)
    got = run(ds)
    assert got.tolist() == [2.25]
    ds = synth.pack([np.array([0.5, 1.0, 2.0]), np.array([-1.0])], "tiny2", -1)
    assert run(ds, kernel="wave").tolist() == [2.25 + 4.0 + 9.0]


# ---------------------------------------------------------------- invariants

def test_identical_series_give_exact_zero():
    rng = np.random.default_rng(11)
    base = [synth.random_walk(rng, 96) for _ in range(40)]
    series = base + base  # series s and s+40 are identical
    for kernel in ("lane", "wave"):
        ds = synth.pack(series, "dup", 9)
        got = run(ds, kernel=kernel)
        k = condensed(np.arange(40), np.arange(40) + 40, 80)
        assert np.all(got[k] == 0.0), kernel
        assert np.all(got[np.setdiff1d(np.arange(len(got)), k)] > 0.0)


@pytest.mark.parametrize("kernel", ["lane", "wave"])
def test_symmetry_bitwise(kernel):
    ds = synth.small_random(seed=3, N=90, len_lo=50, len_hi=50, window=6)
    rev = synth.pack([ds.series(s).astype(np.float64) for s in range(ds.N)][::-1], "rev", 6)
    a = run(ds, kernel=kernel)
    b = run(rev, kernel=kernel)
    pi, pj = oracle.all_pairs_list(ds.N)
    assert np.array_equal(a, b[condensed(ds.N - 1 - pj, ds.N - 1 - pi, ds.N)])


def test_window_monotone_bitwise():
    base = synth.small_random(seed=4, N=40, len_lo=80, len_hi=80)
    prev = None
    for w in [0, 1, 2, 5, 10, 30, 63, -1]:
        ds = synth.pack([base.series(s).astype(np.float64) for s in range(base.N)], "m", w)
        got = run(ds, kernel="wave" if w > 63 or w < 0 else "auto")
        if prev is not None:
            assert np.all(got <= prev), w
        prev = got


# ---------------------------------------------------------------- full-size workloads, sampled

def test_banded_1000x512_sampled():
    ds = synth.config2()
    got = run(ds)
    assert not np.any(np.isnan(got)), "some pair was never written"
    pi, pj = sample_pairs(ds.N, 3000, 1)
    assert_close(got[condensed(pi, pj, ds.N)], oracle_pairs(ds, pi, pj), what="1000x512 w=51")


def test_many_short_8000x256_sampled():
    ds = synth.config5()
    got = run(ds)
    assert not np.any(np.isnan(got)), "some pair was never written"
    pi, pj = sample_pairs(ds.N, 3000, 2)
    assert_close(got[condensed(pi, pj, ds.N)], oracle_pairs(ds, pi, pj), what="8000x256 w=25")


@pytest.mark.parametrize("dtype,accum", [("f32", "plain"), ("f32", "kahan"), ("f32", "fp64"),
                                         ("bf16", "kahan"), ("f16", "kahan"), ("bf16", "plain")])
def test_long_series_precision_modes(dtype, accum):
    ds = synth.config3(dtype=dtype, N=500)
    got = run(ds, accum=accum)
    pi, pj = sample_pairs(ds.N, 24, 3)
    ref = oracle_pairs(ds, pi, pj)
    g = got[condensed(pi, pj, ds.N)]
    if accum == "fp64":
        assert np.array_equal(g, ref.astype(np.float32)), "FP64 mode must equal the oracle rounded to FP32"
    else:
        # 16-bit inputs with plain FP32 sums: 1e-3; FP32 inputs, or any input with compensated sums: 1e-5
        tol = REL_TOL_16BIT_PLAIN if (dtype != "f32" and accum == "plain") else REL_TOL
        assert_close(g, ref, tol=tol, what="500x4096 %s %s" % (dtype, accum))


# ---------------------------------------------------------------- cyclic banded kernel

CYCLIC_H = [1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 24, 28, 32]


def _cyclic_band_limit(H):
    # widest band b for which a lane can take block q+64 after block q: 64(H+1) >= 2b+H
    return (64 * (H + 1) - H) // 2


def _run_plan(ds, **kw):
    plan, series, outs = _plan_for([ds], **kw)
    plan.execute()
    torch.cuda.synchronize()
    info = plan.info()
    got = outs[0].cpu().numpy()[:ds.n_pairs]
    plan.destroy()
    return got, info


def band_edge_pairs(rng, lengths, b):
    """Pairs (x, y) of equal length whose cheapest path runs along the band edge
    i - j = b: x_i = y_max(0, i-b), so that path costs nothing."""
    series = []
    for n in lengths:
        v = synth.random_walk(rng, int(n))
        series.append(v[np.maximum(0, np.arange(n) - b)])
        series.append(v)
    return series


@pytest.mark.parametrize("H", CYCLIC_H)
def test_cyclic_kernel_each_block_height(H):
    _gpu()
    bmax = _cyclic_band_limit(H)
    lo = 64 * H + 30  # more than 64 blocks of H rows: every lane takes several blocks
    rng = np.random.default_rng(700 + H)
    edge = band_edge_pairs(rng, [lo, lo + 7, lo + H + 1], bmax)
    cases = [
        # optimal paths along the band edge, band at the lane-reuse limit
        synth.pack(edge, "edge%d" % H, bmax),
        # band exactly at the lane-reuse limit (|n-m| <= bmax/2 <= w = bmax)
        synth.small_random(seed=300 + H, N=8, len_lo=lo, len_hi=lo + bmax // 2, window=bmax),
        # band well inside the limit, ragged last block
        synth.small_random(seed=400 + H, N=8, len_lo=lo + 1, len_hi=lo + bmax // 3, window=bmax // 3),
        # at most 64 blocks: any band width, lengths from 2 points up
        synth.small_random(seed=500 + H, N=12, len_lo=2, len_hi=64 * H, window=3 * H + 1),
        # two lane cycles with |n-m| near the band limit: windows clipped at
        # the last column on lanes that still take another block
        synth.pack([synth.random_walk(rng, L) for L in
                    (128 * H, 128 * H - bmax + 4, 128 * H - 2, 128 * H - bmax + 2, 128 * H - 1, 128 * H - bmax + 1)],
                   "clip%d" % H, bmax),
    ]
    for k, ds in enumerate(cases):
        got, info = _run_plan(ds, kernel="cyclic", rows_per_lane=H)
        pi, pj = oracle.all_pairs_list(ds.N)
        L = ds.lengths.astype(np.int64)
        bands = [max(ds.window, abs(int(L[a]) - int(L[b]))) for a, b in zip(pi, pj)]
        windowed = sum(1 for (a, b), bb in zip(zip(pi, pj), bands) if bb < max(L[a], L[b]) - 1)
        assert info["n_cyclic_items"] == windowed, (k, info)
        # same per-cell arithmetic as the strip kernel: results agree bit for bit
        wave = run(ds, kernel="wave")
        assert np.array_equal(got, wave), "cyclic H=%d case %d differs from the strip kernel" % (H, k)
        assert_close(got, oracle_pairs(ds, pi, pj), tol=plain_tol(ds), what="cyclic H=%d case %d" % (H, k))


def test_cyclic_long_pairs_and_group_cells():
    # long narrow-band pairs (hundreds of blocks per lane cycle) beside short
    # ones and unequal pairs that fall back to strips; the plan's per-group
    # cell counts add up to its totals
    _gpu()
    rng = np.random.default_rng(4242)
    series = [synth.random_walk(rng, L) for L in (7000, 7010, 6990, 900, 950)]
    ds = synth.pack(series, "long_cyc", 40)
    got, info = _run_plan(ds, kernel="cyclic")
    desc_plan, _, _ = _plan_for([ds], kernel="cyclic")
    groups = desc_plan.describe()["wave_groups"]
    stats = desc_plan.info()
    desc_plan.destroy()
    assert sum(g["band_cells"] for g in groups) == stats["band_cells"]
    assert sum(g["swept_cells"] for g in groups) == stats["computed_cells"]
    pi, pj = oracle.all_pairs_list(ds.N)
    assert_close(got, oracle_pairs(ds, pi, pj), tol=plain_tol(ds), what="cyclic long pairs")
    assert np.array_equal(got, run(ds, kernel="wave"))


@pytest.mark.parametrize("w", [1, 17, 63])
def test_band_edge_paths_all_kernels(w):
    _gpu()
    # equal lengths so that every family applies; cheapest paths hug the band edge
    rng = np.random.default_rng(800 + w)
    ds = synth.pack(band_edge_pairs(rng, [300] * 4, w), "edge", w)
    pi, pj = oracle.all_pairs_list(ds.N)
    ref = oracle_pairs(ds, pi, pj)
    outs = {k: run(ds, kernel=k) for k in ("lane", "wave", "cyclic")}
    for k, got in outs.items():
        assert_close(got, ref, what="band edge w=%d %s" % (w, k))
    assert np.array_equal(outs["lane"], outs["wave"]) and np.array_equal(outs["wave"], outs["cyclic"])


def test_cyclic_band_zero_and_tiny_series():
    _gpu()
    # equal lengths with w=0 (diagonal only), and series of 1..3 points
    rng = np.random.default_rng(77)
    series = [synth.random_walk(rng, 200) for _ in range(5)] + [synth.random_walk(rng, L) for L in (1, 2, 3)]
    for w in (0, 1, 2):
        ds = synth.pack(series, "tiny", w)
        pi, pj = oracle.all_pairs_list(ds.N)
        ref = oracle_pairs(ds, pi, pj)
        for H in (1, 4, 16):
            got, info = _run_plan(ds, kernel="cyclic", rows_per_lane=H)
            assert info["n_cyclic_items"] > 0
            assert_close(got, ref, what="tiny w=%d H=%d" % (w, H))


@pytest.mark.parametrize("frac", [0.05, 0.2])
def test_auto_mixes_strip_and_cyclic(frac):
    _gpu()
    rng = np.random.default_rng(int(frac * 100))
    lens = rng.integers(40, 1400, size=26)
    series = [synth.random_walk(rng, int(L)) for L in lens]
    ds = synth.pack(series, "mix", int(frac * lens.max()))
    got, info = _run_plan(ds)
    assert 0 < info["n_cyclic_items"] < ds.n_pairs, info
    pi, pj = oracle.all_pairs_list(ds.N)
    assert_close(got, oracle_pairs(ds, pi, pj), what="auto mix %.2f" % frac)
    assert np.array_equal(got, run(ds, kernel="wave"))


PLAIN_STRIP_H = [1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64]


@pytest.mark.parametrize("H", PLAIN_STRIP_H)
def test_every_plain_strip_height(H):
    # one-wavefront strips of every instantiated height, with and without a
    # window (two-column sweep / one-column sweep with window events or
    # per-cell tests); the longest series fills the last lanes raggedly
    _gpu()
    for window in (-1, 9):
        ds = synth.small_random(seed=900 + H, N=7, len_lo=max(1, 64 * (H - 1) - 5), len_hi=64 * H, window=window)
        got, info = _run_plan(ds, kernel="wave", rows_per_lane=H)
        pi, pj = oracle.all_pairs_list(ds.N)
        assert_close(got, oracle_pairs(ds, pi, pj), tol=plain_tol(ds), what="strip H=%d w=%d" % (H, window))


@pytest.mark.parametrize("H", [2, 12, 48])
def test_wave_kernel_forced_rows_per_lane(H):
    # a forced strip height gives the same bits as the automatic choice
    ds = synth.small_random(seed=600 + H, N=14, len_lo=1, len_hi=64 * H, window=25)
    assert np.array_equal(run(ds, kernel="wave", rows_per_lane=H), run(ds, kernel="wave"))


# ---------------------------------------------------------------- pair lists

def _random_pairs(rng, N, P):
    i = rng.integers(0, N, size=P)
    j = rng.integers(0, N, size=P)
    pairs = np.stack([i, j], axis=1).astype(np.int32)
    pairs[:3] = [[0, 0], [N - 1, 0], [0, N - 1]]  # a self pair and one pair in both orders
    pairs[3] = pairs[4]                          # a duplicate
    return pairs


@pytest.mark.parametrize("window", [-1, 9, 60])
def test_pair_list_ragged_lengths(window):
    # wavefront kernels (strip and cyclic) on an explicit, unordered pair list
    B = _gpu()
    ds = synth.small_random(seed=700 + max(window, 0), N=60, len_lo=20, len_hi=900, window=window)
    pairs = _random_pairs(np.random.default_rng(1), ds.N, 700)
    got = B.pairs_of(ds, pairs).cpu().numpy()
    ref = oracle_pairs(ds, pairs[:, 0], pairs[:, 1])
    assert_close(got, ref, what="pair list w=%d" % window)
    assert got[0] == 0.0 and got[1] == got[2] and got[3] == got[4]


def test_pair_list_medoids_on_lane_kernel():
    # every series against 5 medoids: tiles of 64 partners around each medoid on
    # the lane-band kernel, bit for bit the values of the all-pairs plan
    from paper_2307_04904_amd import binding as B
    _gpu()
    ds = synth.small_random(seed=71, N=300, len_lo=96, len_hi=96, window=12)
    medoids = [3, 77, 150, 151, 299]
    pairs = np.array([[i, m] for m in medoids for i in range(ds.N)], dtype=np.int32)
    series = B.device_series(ds)
    out = torch.full((len(pairs),), float("nan"), device="cuda")
    plan = B.PairPlan(series, ds.lengths, ds.offsets, ds.window, pairs, out, timing=True)
    for rep in range(2):
        out.fill_(float("nan"))
        plan.execute()
        torch.cuda.synchronize()
    info = plan.info()
    plan.destroy()
    got = out.cpu().numpy()
    assert info["n_wave_items"] == 0 and info["n_lane_items"] == len(medoids) * ((ds.N + 63) // 64)
    full = run(ds)
    self_pair = pairs[:, 0] == pairs[:, 1]
    assert np.all(got[self_pair] == 0.0)
    k = condensed(np.minimum(pairs[:, 0], pairs[:, 1])[~self_pair], np.maximum(pairs[:, 0], pairs[:, 1])[~self_pair],
                  ds.N)
    assert np.array_equal(got[~self_pair], full[k])
    sel = np.random.default_rng(2).choice(len(pairs), 200, replace=False)
    assert_close(got[sel], oracle_pairs(ds, pairs[sel, 0], pairs[sel, 1]), what="medoid pairs")


# ---------------------------------------------------------------- batched plans, graph capture

def _plan_for(dsets, **kw):
    from paper_2307_04904_amd import binding as B
    series = [B.device_series(ds) for ds in dsets]
    outs = [torch.full((max(1, ds.n_pairs),), float("nan"), device="cuda") for ds in dsets]
    plan = B.Plan([(s, ds.lengths, ds.offsets, ds.window, o) for s, ds, o in zip(series, dsets, outs)], **kw)
    return plan, series, outs


def test_batched_uneven_datasets_sampled():
    _gpu()
    dsets = synth.config4()
    plan, series, outs = _plan_for(dsets)
    plan.execute()
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    for d in rng.choice(len(dsets), size=10, replace=False):
        ds = dsets[d]
        got = outs[d].cpu().numpy()
        assert not np.any(np.isnan(got[:ds.n_pairs])), "dataset %d: some pair was never written" % d
        pi, pj = sample_pairs(ds.N, 60, int(d))
        assert_close(got[condensed(pi, pj, ds.N)], oracle_pairs(ds, pi, pj), what="batched dataset %d" % d)
    plan.destroy()


def test_plan_reexecute_with_new_values():
    _gpu()
    ds = synth.small_random(seed=31, N=60, len_lo=70, len_hi=130, window=12)
    plan, series, outs = _plan_for([ds], timing=True)
    pi, pj = oracle.all_pairs_list(ds.N)
    for rep in range(3):
        vals = (ds.values * (1.0 + 0.5 * rep)).astype(np.float32)
        series[0].copy_(torch.from_numpy(vals))
        outs[0].fill_(float("nan"))
        plan.execute()
        assert plan.last_kernel_ms() > 0.0
        ds2 = synth.Dataset("rep", vals, ds.offsets, ds.lengths, ds.window)
        assert_close(outs[0].cpu().numpy(), oracle_pairs(ds2, pi, pj), what="re-execute %d" % rep)
    plan.destroy()


@pytest.mark.parametrize("accum", ["plain", "kahan"])
def test_queue_and_hardware_dispatch_agree(accum):
    # lane-band, strip (one and several wavefronts per pair) and cyclic groups,
    # each launched as resident workgroups pulling from the device queue or as
    # one workgroup per item: the same items give the same bits
    _gpu()
    dsets = [synth.small_random(seed=51, N=90, len_lo=80, len_hi=80, window=7),
             synth.small_random(seed=52, N=40, len_lo=30, len_hi=700, window=25),
             synth.small_random(seed=53, N=12, len_lo=1100, len_hi=1400, window=-1)]
    got = {}
    for q in (True, False):
        plan, series, outs = _plan_for(dsets, accum=accum, queue=q)
        for rep in range(2):  # the queue counters are reset by every execute
            for o in outs:
                o.fill_(float("nan"))
            plan.execute()
            torch.cuda.synchronize()
        got[q] = [o.cpu().numpy()[:ds.n_pairs] for o, ds in zip(outs, dsets)]
        plan.destroy()
    for d, ds in enumerate(dsets):
        assert not np.any(np.isnan(got[True][d])), "dataset %d: a pair was never written" % d
        assert np.array_equal(got[True][d], got[False][d]), "dataset %d" % d
    pi, pj = sample_pairs(dsets[1].N, 40, 5)
    assert_close(got[True][1][condensed(pi, pj, dsets[1].N)], oracle_pairs(dsets[1], pi, pj),
                 what="queue dispatch " + accum)


def test_autotuned_plan_matches_cost_model_plan():
    # the tuner only changes which kernel instance runs a pair; every wavefront
    # instance computes the same bits, so the results must not change
    _gpu()
    dsets = [synth.small_random(seed=61, N=40, len_lo=60, len_hi=1300, window=30),
             synth.small_random(seed=62, N=30, len_lo=200, len_hi=900, window=-1),
             synth.small_random(seed=63, N=60, len_lo=50, len_hi=50, window=5)]
    got = {}
    for tune in (False, True):
        plan, series, outs = _plan_for(dsets, autotune=tune)
        for o in outs:
            o.fill_(float("nan"))
        plan.execute()
        torch.cuda.synchronize()
        got[tune] = [o.cpu().numpy()[:ds.n_pairs] for o, ds in zip(outs, dsets)]
        info, desc = plan.info(), plan.describe()
        plan.destroy()
    assert info["n_tuned_buckets"] == len(desc["tuned"]) > 0
    for b in desc["tuned"]:
        assert b["chosen"] in b["us_per_pair"] and b["model"] in b["us_per_pair"]
        assert min(b["us_per_pair"].values()) == b["us_per_pair"][b["chosen"]] > 0
    assert sum(g["items"] for g in desc["wave_groups"]) == dsets[0].n_pairs + dsets[1].n_pairs
    for d, ds in enumerate(dsets):
        assert np.array_equal(got[True][d], got[False][d]), "dataset %d" % d
    pi, pj = sample_pairs(dsets[0].N, 50, 8)
    assert_close(got[True][0][condensed(pi, pj, dsets[0].N)], oracle_pairs(dsets[0], pi, pj), what="autotuned")


def test_plan_replayed_from_hip_graph():
    _gpu()
    dsets = [synth.small_random(seed=41, N=50, len_lo=64, len_hi=64, window=9),
             synth.small_random(seed=42, N=30, len_lo=20, len_hi=300, window=-1),
             synth.small_random(seed=43, N=30, len_lo=100, len_hi=900, window=40)]
    plan, series, outs = _plan_for(dsets)
    plan.execute()
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for o in outs:
            o.fill_(float("nan"))
        with torch.cuda.graph(g, stream=s):
            plan.execute(s)
    torch.cuda.synchronize()
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), "replay %d differs from the eager result" % rep
    plan.destroy()
