"""Seeded random datasets through every kernel family, accumulation mode and
storage type, against the FP64 oracle (through the C ABI).

Each case draws the series count, a length range (from one point up to past
one wavefront's 64-row capacity), a window (none, zero, narrow, wide) and
optionally equal lengths, so the planner's choices -- lane-band tiles, strip
heights with and without window events, cyclic block heights -- and the
ragged edges of each are exercised together.  The tolerances are the ones of
the parity tests: 1e-5 for FP32 inputs under the default accumulation (and
under rebased or Kahan sums) at every path length, 1e-3 for 16-bit inputs;
FP64 mode bit-exact with the oracle rounded once; explicitly plain FP32 sums
1e-5 up to 2048-cell paths and 1e-4 beyond, and all families of one dataset
agree bit for bit with them."""
import numpy as np
import pytest

import oracle
from paper_2307_04904_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_CASES = 24


def _gpu():
    from paper_2307_04904_amd import binding
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return binding


def _case(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 11))
    hi = int(rng.choice([8, 70, 300, 900, 1600]))
    lo = int(rng.integers(1, hi + 1))
    equal = rng.random() < 0.3
    lens = np.full(N, hi) if equal else rng.integers(lo, hi + 1, size=N)
    window = int(rng.choice([-1, 0, 1 + int(rng.integers(0, 12)), max(1, hi // 10), hi // 3]))
    series = [synth.random_walk(rng, int(L)) for L in lens]
    ds = synth.pack(series, "fuzz%d" % seed, window)
    dtype = str(rng.choice(["f32", "f32", "bf16", "f16"]))
    return synth.with_dtype(ds, dtype) if dtype != "f32" else ds, dtype


def _tol(ds, dtype, accum):
    if dtype != "f32":
        return 1e-3
    if accum != "plain":
        return 1e-5
    L = np.sort(np.asarray(ds.lengths, dtype=np.int64))
    return 1e-5 if int(L[-1] + L[-2] - 1) <= 2048 else 1e-4


def _check(got, ref, tol, what):
    got = np.asarray(got, dtype=np.float64)
    assert np.all(np.isfinite(got)), what + ": non-finite output"
    zero = ref == 0.0
    assert np.all(got[zero] == 0.0), what + ": reference 0 not reproduced exactly"
    rel = np.abs(got[~zero] - ref[~zero]) / ref[~zero]
    assert rel.size == 0 or rel.max() <= tol, "%s: max rel err %.3e > %.1e" % (what, rel.max(), tol)


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_dataset_every_family(seed):
    B = _gpu()
    ds, dtype = _case(31337 + seed)
    print("fuzz seed=%d N=%d lengths=%d..%d window=%d dtype=%s" % (seed, ds.N, ds.lengths.min(), ds.lengths.max(),
                                                                    ds.window, dtype), flush=True)
    pi, pj = oracle.all_pairs_list(ds.N)
    ref, _ = oracle.dtw_pairs(synth.stored_as_f64(ds), ds.offsets, ds.lengths, pi, pj, ds.window)
    equal = bool(np.all(ds.lengths == ds.lengths[0]))
    narrow = ds.window >= 0 and 2 * ds.window + 1 <= 127
    plain = {}
    for kernel in ["auto", "wave", "cyclic"] + (["lane"] if equal and narrow else []):
        got = B.pairwise(ds, kernel=kernel).cpu().numpy()  # default accumulation
        _check(got, ref, _tol(ds, dtype, "auto"), "seed %d %s default" % (seed, kernel))
        got = B.pairwise(ds, kernel=kernel, accum="rebased").cpu().numpy()
        _check(got, ref, _tol(ds, dtype, "rebased"), "seed %d %s rebased" % (seed, kernel))
        got = B.pairwise(ds, kernel=kernel, accum="plain").cpu().numpy()
        _check(got, ref, _tol(ds, dtype, "plain"), "seed %d %s plain" % (seed, kernel))
        plain[kernel] = got
    first = plain["wave"]
    for kernel, got in plain.items():
        assert np.array_equal(got, first), "seed %d: %s differs from the strip kernel" % (seed, kernel)
    kahan = B.pairwise(ds, accum="kahan").cpu().numpy()
    _check(kahan, ref, _tol(ds, dtype, "kahan"), "seed %d kahan" % seed)
    f64 = B.pairwise(ds, accum="fp64").cpu().numpy()
    assert np.array_equal(f64, ref.astype(np.float32)), "seed %d: fp64 mode is not the oracle rounded once" % seed
