"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol the header declares, and rejects bad arguments on the host before any
HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2307_04904_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dtwmi.h")

FAKE_DEV = 0x1000  # never dereferenced: validation fails first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(dtw_\w+)\s*\(", text, flags=re.M)))


def test_header_and_exports_agree():
    names = declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTED)


def test_version():
    assert B.dtw_version() == 100


@pytest.mark.parametrize("n,m,w", [(512, 512, 51), (256, 256, 25), (4096, 4096, -1), (64, 64, -1),
                                   (100, 300, 0), (300, 100, 17), (1, 1, 0), (1, 50, 3), (2048, 64, 102)])
def test_band_cells_matches_oracle(n, m, w):
    assert B.dtw_band_cells(n, m, w) == oracle.band_cells(n, m, w)


def test_band_cells_sweep():
    rng = np.random.default_rng(0)
    for _ in range(300):
        n, m = rng.integers(1, 200, size=2)
        w = int(rng.integers(-1, 220))
        assert B.dtw_band_cells(n, m, w) == oracle.band_cells(n, m, w)


def _call_ex(lengths, offsets, N=None, window=-1, series=FAKE_DEV, out=FAKE_DEV, dtype=0, accum=0, kernel=0, flags=0,
             k_range=(0, 0), pairs_per_wave=0):
    lib = B.load()
    ln = np.ascontiguousarray(lengths, dtype=np.int32)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    d = B.dtw_dataset()
    d.series = ctypes.c_void_p(series)
    d.lengths = ln.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if lengths is not None else None
    d.offsets = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if offsets is not None else None
    d.N = len(ln) if N is None else N
    d.window = window
    d.out_condensed = ctypes.c_void_p(out)
    o = B.dtw_options()
    o.dtype, o.accum, o.kernel, o.flags = dtype, accum, kernel, flags
    o.k_begin, o.k_end = k_range
    o.pairs_per_wave = pairs_per_wave
    rc = lib.dtw_pairwise_ex(ctypes.byref(d), ctypes.byref(o))
    return rc, B.dtw_last_error()


def test_invalid_arguments_rejected_on_host():
    ok_len, ok_off = [4, 4, 4], [0, 4, 8]
    assert _call_ex(ok_len, ok_off, N=-1)[0] == B.DTW_ERR_INVALID_ARG
    assert _call_ex([4, 0, 4], ok_off)[0] == B.DTW_ERR_INVALID_ARG
    assert _call_ex(ok_len, [0, -4, 8])[0] == B.DTW_ERR_INVALID_ARG
    rc, msg = _call_ex(ok_len, ok_off, series=0)
    assert rc == B.DTW_ERR_INVALID_ARG and "series" in msg
    rc, msg = _call_ex(ok_len, ok_off, out=0)
    assert rc == B.DTW_ERR_INVALID_ARG and "out_condensed" in msg
    assert _call_ex(ok_len, ok_off, dtype=7)[0] == B.DTW_ERR_INVALID_ARG
    assert _call_ex(ok_len, ok_off, accum=5)[0] == B.DTW_ERR_INVALID_ARG
    assert _call_ex(ok_len, ok_off, accum=-1)[0] == B.DTW_ERR_INVALID_ARG
    assert _call_ex(ok_len, ok_off, kernel=9)[0] == B.DTW_ERR_INVALID_ARG
    assert _call_ex(ok_len, ok_off, flags=8)[0] == B.DTW_ERR_INVALID_ARG
    for acc in (B.ACCUM["kahan"], B.ACCUM["fp64"]):  # the cyclic kernel has the plain FP32 cell only
        assert _call_ex(ok_len, ok_off, kernel=3, accum=acc)[0] == B.DTW_ERR_UNSUPPORTED
    lib = B.load()
    assert lib.dtw_pairwise_ex(None, None) == B.DTW_ERR_INVALID_ARG
    assert lib.dtw_plan_destroy(None) == B.DTW_ERR_INVALID_ARG
    assert lib.dtw_plan_execute(None, None) == B.DTW_ERR_INVALID_ARG
    assert lib.dtw_band_cells(3, 3, 0, None) == B.DTW_ERR_INVALID_ARG
    need = ctypes.c_int64()
    assert lib.dtw_plan_describe(None, None, ctypes.c_int64(0), ctypes.byref(need)) == B.DTW_ERR_INVALID_ARG
    assert _call_ex(ok_len, ok_off, flags=16)[0] == B.DTW_ERR_INVALID_ARG


def _call_pairs(pairs, N=4, out=FAKE_DEV, series=FAKE_DEV):
    lib = B.load()
    ln = np.full(N, 5, dtype=np.int32)
    off = np.arange(N, dtype=np.int64) * 5
    d = B.dtw_dataset()
    d.series = ctypes.c_void_p(series)
    d.lengths = ln.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.offsets = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    d.N, d.window, d.out_condensed = N, -1, None
    arr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    ptr = arr.ctypes.data_as(ctypes.POINTER(B.dtw_pair)) if len(arr) else None
    rc = lib.dtw_pairs(ctypes.byref(d), ptr, ctypes.c_int64(len(arr)), ctypes.c_void_p(out), None)
    return rc, B.dtw_last_error()


def test_pair_list_validation_on_host():
    assert _call_pairs([])[0] == B.DTW_OK  # nothing to do, no HIP call
    rc, msg = _call_pairs([[0, 1], [2, 4]])
    assert rc == B.DTW_ERR_INVALID_ARG and "pairs[1]" in msg
    assert _call_pairs([[0, -1]])[0] == B.DTW_ERR_INVALID_ARG
    assert _call_pairs([[0, 1]], out=0)[0] == B.DTW_ERR_INVALID_ARG
    assert _call_pairs([[0, 1]], series=0)[0] == B.DTW_ERR_INVALID_ARG
    lib = B.load()
    assert lib.dtw_plan_create_pairs(None, None, None, ctypes.c_int64(0), None, None) == B.DTW_ERR_INVALID_ARG


def test_cluster_score_arguments_rejected_on_host():
    lib = B.load()
    mean, tot = ctypes.c_double(), ctypes.c_double()
    dev = ctypes.c_void_p(FAKE_DEV)
    assert lib.dtw_silhouette(None, 10, dev, 2, None, ctypes.byref(mean), None) == B.DTW_ERR_INVALID_ARG
    assert lib.dtw_silhouette(dev, 1, dev, 2, None, ctypes.byref(mean), None) == B.DTW_ERR_INVALID_ARG
    assert lib.dtw_silhouette(dev, 10, dev, 1, None, ctypes.byref(mean), None) == B.DTW_ERR_INVALID_ARG
    assert lib.dtw_silhouette(dev, 10, dev, 65, None, ctypes.byref(mean), None) == B.DTW_ERR_UNSUPPORTED
    assert lib.dtw_cluster_cost(dev, 10, None, dev, 2, None, ctypes.byref(tot), None) == B.DTW_ERR_INVALID_ARG
    assert lib.dtw_assign(dev, 10, dev, 11, dev, None, ctypes.byref(tot), None) == B.DTW_ERR_INVALID_ARG
    assert lib.dtw_assign(dev, 10, dev, 2, None, None, ctypes.byref(tot), None) == B.DTW_ERR_INVALID_ARG


def test_path_arguments_rejected_on_host():
    lib = B.load()
    dev = ctypes.c_void_p(FAKE_DEV)
    ln, cost = ctypes.c_int64(), ctypes.c_float()

    def call(x=dev, n=4, y=dev, m=4, path=dev, length=True, c=True):
        rc = lib.dtw_path(x, n, y, m, -1, path, ctypes.byref(ln) if length else None,
                          ctypes.byref(cost) if c else None, None, None)
        return rc, B.dtw_last_error()

    assert call(x=None)[0] == B.DTW_ERR_INVALID_ARG
    assert call(path=None)[0] == B.DTW_ERR_INVALID_ARG
    assert call(length=False)[0] == B.DTW_ERR_INVALID_ARG
    assert call(c=False)[0] == B.DTW_ERR_INVALID_ARG
    assert call(n=0)[0] == B.DTW_ERR_INVALID_ARG
    assert call(m=-1)[0] == B.DTW_ERR_INVALID_ARG
    rc, msg = call(n=32769, m=40000)
    assert rc == B.DTW_ERR_UNSUPPORTED and "32768" in msg


def test_fewer_than_two_series_is_a_no_op():
    # no HIP call is made: this passes on a machine without a GPU
    assert _call_ex([], [], series=0, out=0)[0] == B.DTW_OK
    assert _call_ex([5], [0], series=0, out=0)[0] == B.DTW_OK


def test_unsupported_requests_rejected_on_host():
    # forcing the lane-band kernel on unequal lengths
    rc, msg = _call_ex([4, 5, 4], [0, 4, 9], kernel=1)
    assert rc == B.DTW_ERR_UNSUPPORTED and "lane-band" in msg
    # lane-band kernel with Kahan or FP64 accumulation
    assert _call_ex([4, 4], [0, 4], kernel=1, accum=B.ACCUM["kahan"])[0] == B.DTW_ERR_UNSUPPORTED
    assert _call_ex([4, 4], [0, 4], kernel=1, accum=B.ACCUM["fp64"])[0] == B.DTW_ERR_UNSUPPORTED
    # (pairs longer than one workgroup's rows are swept in row passes: no
    # length limit to reject here; the GPU tests cover them)


def test_accumulation_enum_matches_header():
    text = open(HEADER).read()
    for name, val in B.ACCUM.items():
        assert re.search(r"DTW_ACC_%s\s*=\s*%d\b" % (name.upper(), val), text), name
    # a zero-initialised dtw_options asks for AUTO accumulation
    assert B.ACCUM["auto"] == 0


def test_output_range_validated_on_host():
    ok_len, ok_off = [4, 4, 4], [0, 4, 8]
    rc, msg = _call_ex(ok_len, ok_off, k_range=(-1, 0))
    assert rc == B.DTW_ERR_INVALID_ARG and "range" in msg
    rc, msg = _call_ex(ok_len, ok_off, k_range=(2, 1))
    assert rc == B.DTW_ERR_INVALID_ARG and "range" in msg
    # the options struct carries the range after the stream pointer
    assert B.dtw_options.k_begin.offset == 32 and B.dtw_options.k_end.offset == 40
    assert ctypes.sizeof(B.dtw_options) == 48


def test_pairs_per_wave_validated_on_host():
    ok_len, ok_off = [4, 4, 4], [0, 4, 8]
    for bad in (-1, 1, 3, 32, 65):
        rc, msg = _call_ex(ok_len, ok_off, pairs_per_wave=bad)
        assert rc == B.DTW_ERR_INVALID_ARG and "pairs_per_wave" in msg
    # between rows_per_lane and the stream pointer, where the struct had padding
    assert B.dtw_options.pairs_per_wave.offset == 20 and B.dtw_options.stream.offset == 24
    text = open(HEADER).read()
    assert text.index("int32_t rows_per_lane;") < text.index("int32_t pairs_per_wave;") < text.index("void *stream;")


def test_series_length_limit_on_host():
    rc, msg = _call_ex([5, (1 << 28) + 1], [0, 5])
    assert rc == B.DTW_ERR_UNSUPPORTED and "exceeds" in msg


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(B.DtwError):
        B.load(str(tmp_path / "missing.so"))
