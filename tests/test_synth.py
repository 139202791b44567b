"""Seeded generators: reproducible, right shapes, exact 16-bit casts."""
import numpy as np
import pytest

from paper_2307_04904_amd import synth


def test_config1_shape_and_reproducible():
    a = synth.config1()
    b = synth.config1()
    assert a.N == 20 and a.n_pairs == 190 and a.window == -1
    assert np.all(a.lengths == 64) and a.values.dtype == np.float32
    assert np.array_equal(a.values, b.values)
    for s in range(a.N):
        v = a.series(s).astype(np.float64)
        assert abs(v.mean()) < 1e-6 and abs(v.std() - 1.0) < 1e-5


def test_config2_and_5_headers():
    c2 = synth.config2()
    assert c2.N == 1000 and c2.window == 51 and np.all(c2.lengths == 512)
    assert c2.n_pairs == 499500
    c5 = synth.config5(N=300)
    assert c5.window == 25 and np.all(c5.lengths == 256)


def test_config4_ranges():
    ds = synth.config4(n_datasets=6)
    assert len(ds) == 6
    for d in ds:
        assert 10 <= d.N <= 400
        assert d.lengths.min() >= 64 and d.lengths.max() <= 2048
        assert d.window == -1 or d.window == int(np.floor(d.meta["window_fraction"] * d.lengths.max()))
    # the default seed is the workload's own; another seed draws another instance of the recipe
    same = synth.config4(n_datasets=6, seed=synth.SEEDS["c4"])
    assert all(np.array_equal(a.values, b.values) and a.window == b.window for a, b in zip(ds, same))
    other = synth.config4(n_datasets=6, seed=1)
    assert [d.N for d in other] != [d.N for d in ds]
    assert all(10 <= d.N <= 400 and 64 <= d.lengths.min() and d.lengths.max() <= 2048 for d in other)


def test_bf16_and_f16_are_rne_casts():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(10000) * 3).astype(np.float32)
    bits = synth.f32_to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(bits, ref)
    back = synth.bf16_bits_to_f32(bits)
    assert np.array_equal(back, torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy())
    ds = synth.config3(dtype="f16", N=3, L=64)
    assert ds.values.dtype == np.float16
