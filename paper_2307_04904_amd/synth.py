"""Seeded synthetic inputs for the all-pairs DTW workloads.

This module only makes input data: it holds none of the DTW arithmetic and
imports neither the GPU library nor the oracle, so that both can be fed the
very same stored arrays.

Every generator draws with ``numpy.random.Generator(PCG64(seed))`` in FP64,
z-normalises each series (population standard deviation) in FP64 and rounds
to FP32 with round-to-nearest-even.  16-bit forms are RNE casts of that FP32
array.  The series shapes stand in for the UCR archive datasets the paper
benchmarks on (Performance comparison section): random walks of UCR-like
counts and lengths, plus a shape-class mixture for the many-short-series case.

A dataset is a ragged concatenation: ``values`` (1-D), ``offsets`` (int64,
start of each series) and ``lengths`` (int32), plus an integer ``window``
(-1 = no window).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FULL = -1


@dataclass
class Dataset:
    name: str
    values: np.ndarray          # float32 (or uint16 bf16 bits / float16 for 16-bit forms)
    offsets: np.ndarray         # int64
    lengths: np.ndarray         # int32
    window: int = FULL
    dtype: str = "f32"          # "f32" | "bf16" | "f16"
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(len(self.lengths))

    @property
    def n_pairs(self) -> int:
        return self.N * (self.N - 1) // 2

    def series(self, s: int) -> np.ndarray:
        o = int(self.offsets[s])
        return self.values[o:o + int(self.lengths[s])]

    def as_f32_values(self) -> np.ndarray:
        """Stored values widened exactly to float32 (identity for f32)."""
        if self.dtype == "bf16":
            return bf16_bits_to_f32(self.values)
        return self.values.astype(np.float32)


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(int(seed)))


def znorm(x: np.ndarray) -> np.ndarray:
    """(x - mean) / std with ddof=0, in float64; a constant series stays zero."""
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean()
    sd = x.std()
    if sd == 0.0:
        return np.zeros_like(x)
    return (x - mu) / sd


def random_walk(rng: np.random.Generator, L: int) -> np.ndarray:
    """x_t = sum of t+1 standard normal steps, z-normalised (float64)."""
    return znorm(np.cumsum(rng.standard_normal(L)))


def pack(series_list, name: str, window: int, meta=None) -> Dataset:
    """Concatenate float64 series into a float32 ragged dataset."""
    lengths = np.array([len(s) for s in series_list], dtype=np.int32)
    offsets = np.zeros(len(series_list), dtype=np.int64)
    if len(series_list) > 1:
        offsets[1:] = np.cumsum(lengths[:-1], dtype=np.int64)
    if len(series_list):
        values = np.concatenate([np.asarray(s, dtype=np.float64) for s in series_list]).astype(np.float32)
    else:
        values = np.zeros(0, dtype=np.float32)
    return Dataset(name=name, values=values, offsets=offsets, lengths=lengths,
                   window=int(window), dtype="f32", meta=dict(meta or {}))


# ---------------------------------------------------------------- 16-bit forms

def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (RNE), returned as raw uint16 bits (finite inputs)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    return ((u + bias) >> 16).astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.ascontiguousarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def with_dtype(ds: Dataset, dtype: str) -> Dataset:
    """The same dataset stored as "f32", "bf16" (uint16 bits) or "f16" (RNE casts of the f32 array)."""
    base = ds.as_f32_values()
    if dtype == "f32":
        vals = base.copy()
    elif dtype == "bf16":
        vals = f32_to_bf16_bits(base)
    elif dtype == "f16":
        vals = base.astype(np.float16)
    else:
        raise ValueError(dtype)
    return Dataset(name=ds.name + ":" + dtype, values=vals, offsets=ds.offsets.copy(),
                   lengths=ds.lengths.copy(), window=ds.window, dtype=dtype, meta=dict(ds.meta))


def stored_as_f64(ds: Dataset) -> np.ndarray:
    """Exact float64 image of the stored values (what both sides must compute on)."""
    if ds.dtype == "bf16":
        return bf16_bits_to_f32(ds.values).astype(np.float64)
    return ds.values.astype(np.float64)


# ---------------------------------------------------------------- workloads

SEEDS = {"c1": 230704901, "c2": 230704902, "c3": 230704903, "c4": 230704904, "c5": 230704905}


def random_walk_dataset(seed, N: int, L: int, window: int, name: str, noise: float = 0.0) -> Dataset:
    rng = _rng(seed)
    out = []
    for _ in range(N):
        s = random_walk(rng, L)
        if noise:
            s = s + noise * rng.standard_normal(L)
        out.append(s)
    return pack(out, name, window, dict(seed=int(seed), N=N, L=L, noise=noise))


def config1() -> Dataset:
    """20 random walks of length 64, no window (the smallest case)."""
    return random_walk_dataset(SEEDS["c1"], 20, 64, FULL, "c1_20x64_full")


def config2() -> Dataset:
    """1000 random walks of length 512, Sakoe-Chiba window 51 (10%)."""
    return random_walk_dataset(SEEDS["c2"], 1000, 512, 51, "c2_1000x512_w51")


def config3(dtype: str = "f32", N: int = 500, L: int = 4096) -> Dataset:
    """500 series of length 4096, random walk plus 0.1 N(0,1) noise after z-normalising, no window."""
    ds = random_walk_dataset(SEEDS["c3"], N, L, FULL, "c3_%dx%d_full" % (N, L), noise=0.1)
    return with_dtype(ds, dtype) if dtype != "f32" else ds


WINDOW_FRACTIONS = (0.0, 0.05, 0.10, 0.20, None)  # None = no window


def config4(n_datasets: int = 64, n_lo: int = 10, n_hi: int = 400, len_lo: int = 64, len_hi: int = 2048,
            seed=None):
    """64 independent datasets of uneven size and uneven series lengths.

    N ~ U{n_lo..n_hi}; every series length ~ U{len_lo..len_hi}; window fraction
    p ~ U{0, 5%, 10%, 20%, none}, turned into w = floor(p * longest length).
    `seed` (default: the workload's own) draws another instance of the recipe.
    """
    children = np.random.SeedSequence(SEEDS["c4"] if seed is None else seed).spawn(n_datasets)
    out = []
    for d, child in enumerate(children):
        rng = _rng(child)
        N = int(rng.integers(n_lo, n_hi + 1))
        lens = rng.integers(len_lo, len_hi + 1, size=N)
        frac = WINDOW_FRACTIONS[int(rng.integers(0, len(WINDOW_FRACTIONS)))]
        w = FULL if frac is None else int(np.floor(frac * int(lens.max())))
        series = [random_walk(rng, int(L)) for L in lens]
        out.append(pack(series, "c4_d%02d" % d, w, dict(window_fraction=frac)))
    return out


def _template(kind: int, cycles: int, L: int) -> np.ndarray:
    phase = cycles * np.arange(L, dtype=np.float64) / L
    if kind == 0:
        return np.sin(2.0 * np.pi * phase)
    if kind == 1:
        return np.where(np.sin(2.0 * np.pi * phase) >= 0.0, 1.0, -1.0)
    return 2.0 * (phase - np.floor(phase)) - 1.0


def config5(N: int = 8000, L: int = 256) -> Dataset:
    """8000 series of length 256, window 25: half random walks, half noisy shape classes.

    Class k in 0..9 uses a sine / square / sawtooth template (k mod 3) with
    1 + k//3 cycles, circularly shifted by U{0..25} samples, plus N(0, 0.2^2).
    """
    rng = _rng(SEEDS["c5"])
    out = []
    for _ in range(N):
        if rng.random() < 0.5:
            out.append(random_walk(rng, L))
        else:
            k = int(rng.integers(0, 10))
            shift = int(rng.integers(0, 26))
            s = np.roll(_template(k % 3, 1 + k // 3, L), shift) + rng.normal(0.0, 0.2, L)
            out.append(znorm(s))
    return pack(out, "c5_%dx%d_w25" % (N, L), 25, dict(N=N, L=L))


def small_random(seed: int, N: int, len_lo: int, len_hi: int, window: int = FULL, integer: bool = False) -> Dataset:
    """Small ragged test dataset; integer=True gives small integers (exact sums)."""
    rng = _rng(seed)
    lens = rng.integers(len_lo, len_hi + 1, size=N)
    series = []
    for L in lens:
        if integer:
            series.append(rng.integers(-4, 5, size=int(L)).astype(np.float64))
        else:
            series.append(random_walk(rng, int(L)))
    return pack(series, "rand_s%d" % seed, window)
