"""Thin ctypes binding of libdtwmi.so (declared in include/dtwmi.h).

Argument marshalling only: device buffers are torch tensors on the GPU (their
``data_ptr()`` is passed through), host arrays are numpy arrays, streams are
torch streams.  Every computation happens in the HIP kernels behind the C ABI;
if the library is missing this module raises instead of computing anything.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "libdtwmi.so")

DTW_OK, DTW_ERR_INVALID_ARG, DTW_ERR_UNSUPPORTED, DTW_ERR_OUT_OF_MEMORY, DTW_ERR_HIP = range(5)
DTYPES = {"f32": 0, "bf16": 1, "f16": 2}
ACCUM = {"auto": 0, "plain": 1, "kahan": 2, "fp64": 3, "rebased": 4}
KERNELS = {"auto": 0, "lane": 1, "wave": 2, "cyclic": 3}
DTW_FLAG_TIMING = 1
DTW_FLAG_NO_QUEUE = 2
DTW_FLAG_AUTOTUNE = 4

EXPORTED = ["dtw_pairwise", "dtw_pairwise_ex", "dtw_pairwise_noalloc", "dtw_plan_create", "dtw_plan_execute",
            "dtw_plan_last_kernel_ms", "dtw_plan_info", "dtw_plan_describe", "dtw_plan_destroy", "dtw_band_cells",
            "dtw_plan_create_pairs", "dtw_pairs", "dtw_silhouette", "dtw_cluster_cost", "dtw_assign",
            "dtw_path", "dtw_last_error", "dtw_version"]


class DtwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("dtwmi error %d: %s" % (code, msg))
        self.code = code


class dtw_dataset(ctypes.Structure):
    _fields_ = [("series", ctypes.c_void_p), ("lengths", ctypes.POINTER(ctypes.c_int32)),
                ("offsets", ctypes.POINTER(ctypes.c_int64)), ("N", ctypes.c_int32),
                ("window", ctypes.c_int32), ("out_condensed", ctypes.c_void_p)]


class dtw_options(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("accum", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("rows_per_lane", ctypes.c_int32), ("pairs_per_wave", ctypes.c_int32),
                ("stream", ctypes.c_void_p),
                ("k_begin", ctypes.c_int64), ("k_end", ctypes.c_int64)]


class dtw_pair(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int32), ("j", ctypes.c_int32)]


class dtw_plan_stats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("band_cells", ctypes.c_int64), ("computed_cells", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("n_launches", ctypes.c_int32),
                ("n_lane_items", ctypes.c_int32), ("n_wave_items", ctypes.c_int64),
                ("n_cyclic_items", ctypes.c_int64), ("n_tuned_buckets", ctypes.c_int32),
                ("n_tuned_changed", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libdtwmi.so (raises DtwError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise DtwError(-1, "%s is missing: build it with __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    i32p, i64p = P(ctypes.c_int32), P(ctypes.c_int64)
    lib.dtw_pairwise.argtypes = [ctypes.c_void_p, i32p, i64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    lib.dtw_pairwise_ex.argtypes = [P(dtw_dataset), P(dtw_options)]
    lib.dtw_pairwise_noalloc.argtypes = [P(dtw_dataset), P(dtw_options)]
    lib.dtw_plan_create.argtypes = [P(ctypes.c_void_p), P(dtw_dataset), ctypes.c_int32, P(dtw_options)]
    lib.dtw_plan_execute.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.dtw_plan_last_kernel_ms.argtypes = [ctypes.c_void_p, P(ctypes.c_float)]
    lib.dtw_plan_info.argtypes = [ctypes.c_void_p, P(dtw_plan_stats)]
    lib.dtw_plan_destroy.argtypes = [ctypes.c_void_p]
    lib.dtw_band_cells.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, i64p]
    lib.dtw_last_error.argtypes = []
    lib.dtw_last_error.restype = ctypes.c_char_p
    lib.dtw_version.argtypes = []
    lib.dtw_version.restype = ctypes.c_int32
    for name in EXPORTED:
        if name not in ("dtw_last_error", "dtw_version"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != DTW_OK:
        raise DtwError(rc, dtw_last_error())


def dtw_last_error() -> str:
    return load().dtw_last_error().decode()


def dtw_version() -> int:
    return int(load().dtw_version())


def dtw_band_cells(n: int, m: int, window: int) -> int:
    out = ctypes.c_int64()
    _check(load().dtw_band_cells(int(n), int(m), int(window), ctypes.byref(out)))
    return int(out.value)


def _host_arrays(lengths, offsets):
    ln = np.ascontiguousarray(lengths, dtype=np.int32)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    return ln, off


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _make_dataset(series, lengths, offsets, window, out):
    ln, off = _host_arrays(lengths, offsets)
    d = dtw_dataset()
    d.series = ctypes.c_void_p(series.data_ptr() if series is not None else 0)
    d.lengths = ln.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.offsets = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    d.N = len(ln)
    d.window = int(window)
    d.out_condensed = ctypes.c_void_p(out.data_ptr() if out is not None else 0)
    return d, (ln, off)


def _options(dtype="f32", accum="auto", kernel="auto", flags=0, stream=None, rows_per_lane=0, k_range=(0, 0),
             pairs_per_wave=0):
    o = dtw_options()
    o.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    o.accum = ACCUM[accum] if isinstance(accum, str) else int(accum)
    o.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.flags = int(flags)
    o.rows_per_lane = int(rows_per_lane)
    o.pairs_per_wave = int(pairs_per_wave)
    o.stream = _stream_handle(stream) if stream is not False else ctypes.c_void_p(0)
    o.k_begin, o.k_end = int(k_range[0]), int(k_range[1])
    return o


def dtw_pairwise(series, lengths, offsets, N, window, out_condensed):
    """Short form of the C ABI: FP32 device series, condensed FP32 device output, enqueued on the default stream."""
    ln, off = _host_arrays(lengths, offsets)
    _check(load().dtw_pairwise(ctypes.c_void_p(series.data_ptr()), ln.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(N), int(window),
                               ctypes.c_void_p(out_condensed.data_ptr())))


def dtw_pairwise_noalloc(series, lengths, offsets, window, out_condensed, dtype="f32", accum="auto", kernel="auto",
                         stream=None):
    """The allocation-free entry point (static device workspace), enqueued on `stream`."""
    d, keep = _make_dataset(series, lengths, offsets, window, out_condensed)
    o = _options(dtype, accum, kernel, 0, stream)
    _check(load().dtw_pairwise_noalloc(ctypes.byref(d), ctypes.byref(o)))
    del keep


def dtw_pairwise_ex(series, lengths, offsets, window, out_condensed, dtype="f32", accum="auto", kernel="auto",
                    stream=None, rows_per_lane=0, queue=True, k_range=(0, 0), pairs_per_wave=0):
    """One dataset with options, enqueued on `stream` (None = torch's current stream).

    `series` holds f32, bf16 (as int16/uint16 bits) or f16 values; k_range = (k_begin, k_end) restricts the
    written condensed entries (0, 0 = all)."""
    d, keep = _make_dataset(series, lengths, offsets, window, out_condensed)
    o = _options(dtype, accum, kernel, 0 if queue else DTW_FLAG_NO_QUEUE, stream, rows_per_lane, k_range,
                 pairs_per_wave)
    _check(load().dtw_pairwise_ex(ctypes.byref(d), ctypes.byref(o)))
    del keep


class Plan:
    """dtw_plan_create / execute / destroy for one or more datasets.

    datasets: list of (series_tensor, lengths, offsets, window, out_tensor).
    The tensors must stay alive, at the same address, while the plan exists.
    """

    def __init__(self, datasets, dtype="f32", accum="auto", kernel="auto", timing=False, rows_per_lane=0,
                 queue=True, autotune=False, k_range=(0, 0), pairs_per_wave=0):
        self._lib = load()
        arr = (dtw_dataset * max(1, len(datasets)))()
        self._keep = []
        for k, (series, lengths, offsets, window, out) in enumerate(datasets):
            d, keep = _make_dataset(series, lengths, offsets, window, out)
            arr[k] = d
            self._keep.append((keep, series, out))
        flags = ((DTW_FLAG_TIMING if timing else 0) | (0 if queue else DTW_FLAG_NO_QUEUE)
                 | (DTW_FLAG_AUTOTUNE if autotune else 0))
        o = _options(dtype, accum, kernel, flags, False, rows_per_lane, k_range, pairs_per_wave)
        self._h = ctypes.c_void_p()
        _check(self._lib.dtw_plan_create(ctypes.byref(self._h), arr, len(datasets), ctypes.byref(o)))

    def execute(self, stream=None):
        _check(self._lib.dtw_plan_execute(self._h, _stream_handle(stream)))

    def last_kernel_ms(self) -> float:
        ms = ctypes.c_float()
        _check(self._lib.dtw_plan_last_kernel_ms(self._h, ctypes.byref(ms)))
        return float(ms.value)

    def info(self) -> dict:
        st = dtw_plan_stats()
        _check(self._lib.dtw_plan_info(self._h, ctypes.byref(st)))
        return {name: int(getattr(st, name)) for name, _ in dtw_plan_stats._fields_}

    def describe(self) -> dict:
        """dtw_plan_describe parsed: kernel groups and autotuning measurements."""
        import json
        need = ctypes.c_int64()
        _check(self._lib.dtw_plan_describe(self._h, None, ctypes.c_int64(0), ctypes.byref(need)))
        buf = ctypes.create_string_buffer(int(need.value))
        _check(self._lib.dtw_plan_describe(self._h, buf, ctypes.c_int64(need.value), ctypes.byref(need)))
        return json.loads(buf.value.decode())

    def destroy(self):
        if self._h:
            _check(self._lib.dtw_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _pair_array(pairs):
    """(P, 2) integer pairs as a contiguous int32 array usable as dtw_pair[P]."""
    a = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    return a, a.ctypes.data_as(ctypes.POINTER(dtw_pair))


def dtw_pairs(series, lengths, offsets, window, pairs, out, dtype="f32", accum="auto", kernel="auto",
              stream=None, queue=True, k_range=(0, 0), pairs_per_wave=0):
    """Pair-list evaluation enqueued on `stream`: out[k] = DTW(series pairs[k][0], series pairs[k][1])."""
    d, keep = _make_dataset(series, lengths, offsets, window, None)
    arr, ptr = _pair_array(pairs)
    o = _options(dtype, accum, kernel, 0 if queue else DTW_FLAG_NO_QUEUE, stream, 0, k_range, pairs_per_wave)
    _check(load().dtw_pairs(ctypes.byref(d), ptr, ctypes.c_int64(len(arr)),
                            ctypes.c_void_p(out.data_ptr() if out is not None else 0), ctypes.byref(o)))
    del keep


class PairPlan(Plan):
    """dtw_plan_create_pairs: a plan over an explicit pair list of one dataset."""

    def __init__(self, series, lengths, offsets, window, pairs, out, dtype="f32", accum="auto", kernel="auto",
                 timing=False, queue=True, autotune=False, pairs_per_wave=0):
        self._lib = load()
        d, keep = _make_dataset(series, lengths, offsets, window, None)
        arr, ptr = _pair_array(pairs)
        self._keep = [(keep, series, out, arr)]
        flags = ((DTW_FLAG_TIMING if timing else 0) | (0 if queue else DTW_FLAG_NO_QUEUE)
                 | (DTW_FLAG_AUTOTUNE if autotune else 0))
        o = _options(dtype, accum, kernel, flags, False, pairs_per_wave=pairs_per_wave)
        self._h = ctypes.c_void_p()
        _check(self._lib.dtw_plan_create_pairs(ctypes.byref(self._h), ctypes.byref(d), ptr, ctypes.c_int64(len(arr)),
                                               ctypes.c_void_p(out.data_ptr()), ctypes.byref(o)))


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def silhouette(D, N, labels, K, s_out=None, stream=None):
    """dtw_silhouette: mean silhouette (float) of device int32 labels over the condensed device matrix D."""
    mean = ctypes.c_double()
    _check(load().dtw_silhouette(_dptr(D), int(N), _dptr(labels), int(K), _dptr(s_out), ctypes.byref(mean),
                                 _stream_handle(stream)))
    return float(mean.value)


def cluster_cost(D, N, labels, centroids, stream=None):
    """dtw_cluster_cost: (total, per-cluster list) of a labelling with the given centroid series."""
    K = int(centroids.numel())
    per = (ctypes.c_double * K)()
    tot = ctypes.c_double()
    _check(load().dtw_cluster_cost(_dptr(D), int(N), _dptr(labels), _dptr(centroids), K, per, ctypes.byref(tot),
                                   _stream_handle(stream)))
    return float(tot.value), [float(v) for v in per]


def assign(D, N, centroids, labels_out, stream=None):
    """dtw_assign: nearest-centroid labels into labels_out (device int32); returns (total, per-cluster list)."""
    K = int(centroids.numel())
    per = (ctypes.c_double * K)()
    tot = ctypes.c_double()
    _check(load().dtw_assign(_dptr(D), int(N), _dptr(centroids), K, _dptr(labels_out), per, ctypes.byref(tot),
                             _stream_handle(stream)))
    return float(tot.value), [float(v) for v in per]


def warping_path(x, y, window=-1, path_out=None, C_out=None, stream=None):
    """dtw_path: the optimal warping path of device series x, y.

    Returns (path, cost): path is the leading (L, 2) int32 view of path_out (a
    device tensor of 2*(n+m-1) int32, allocated here if None), cost the float
    c(n, m).  C_out (device float32, n*m) receives the row-major cost matrix.
    """
    import torch
    n, m = int(x.numel()), int(y.numel())
    if path_out is None:
        path_out = torch.empty(2 * (n + m - 1), dtype=torch.int32, device=x.device)
    length, cost = ctypes.c_int64(), ctypes.c_float()
    _check(load().dtw_path(_dptr(x), n, _dptr(y), m, int(window), _dptr(path_out), ctypes.byref(length),
                           ctypes.byref(cost), _dptr(C_out), _stream_handle(stream)))
    return path_out[: 2 * length.value].view(-1, 2), float(cost.value)


def device_series(ds, device="cuda"):
    """Upload a synth.Dataset's stored values as a torch tensor (bf16 kept as raw 16-bit words)."""
    import torch
    v = ds.values
    if ds.dtype == "bf16":
        t = torch.from_numpy(v.view(np.int16).copy())
    elif ds.dtype == "f16":
        t = torch.from_numpy(v.copy())
    else:
        t = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32))
    return t.to(device)


def pairs_of(ds, pairs, accum="auto", kernel="auto", device="cuda", pairs_per_wave=0):
    """DTW of listed pairs of a synth.Dataset on the GPU, as a torch tensor (enqueued on the current stream)."""
    import torch
    series = device_series(ds, device)
    out = torch.full((max(1, len(pairs)),), float("nan"), dtype=torch.float32, device=device)
    dtw_pairs(series, ds.lengths, ds.offsets, ds.window, pairs, out, dtype=ds.dtype, accum=accum, kernel=kernel,
              pairs_per_wave=pairs_per_wave)
    return out[:len(pairs)]


def pairwise(ds, accum="auto", kernel="auto", device="cuda", out=None, rows_per_lane=0, queue=True, k_range=(0, 0),
             pairs_per_wave=0):
    """Condensed DTW matrix of a synth.Dataset on the GPU, as a torch tensor (enqueued on the current stream)."""
    import torch
    series = device_series(ds, device)
    if out is None:
        out = torch.full((max(0, ds.n_pairs),), float("nan"), dtype=torch.float32, device=device)
    dtw_pairwise_ex(series, ds.lengths, ds.offsets, ds.window, out, dtype=ds.dtype, accum=accum, kernel=kernel,
                    rows_per_lane=rows_per_lane, queue=queue, k_range=k_range, pairs_per_wave=pairs_per_wave)
    return out
