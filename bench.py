#!/usr/bin/env python3
"""Throughput of the all-pairs DTW distance matrix on one MI355X.

One step = one evaluation of the whole hot path on the workload's synthetic
input, already resident in HBM: the staging kernel (padded FP32 copy of the
series) and the DP kernels, i.e. one dtw_plan_execute.  The metric is giga
cell updates per second over the admissible (in-window) cells of every pair.

Printed: one JSON line with the value, the roofline of the dominant DP kernel
(FP32 VALU bound, 3 VALU lane-operations per cell: sub, min3, fma), and the
FP64 CPU oracle timed on a bounded sample of the same workload.  The default
run (8000 series of 256 points, window 25, the largest single-matrix
workload) adds, under "extra": the equal-length banded matrix (1000 x 512,
window 51) as the equal-size rate, the 64-dataset batched plan replayed from a
HIP graph with its ratio to that rate (and the same plan autotuned), the
k-medoids pair list on the 1000 x 512 data, the 500 x 4096 long-series matrix
under the default accumulation with its error against the oracle, and the
headline matrix with its series stored as BF16 and as FP16, each with its
error against the oracle on the stored values.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz.  The published FP32 vector peak of 157.3 TFLOP/s
# is 256 CU x 128 lanes x 2 flops (FMA) x 2.4 GHz; counted as VALU
# lane-operations (one FMA, min3 or sub = 1 op) it is 78.64 T op/s.
PEAK_LANE_OPS_T = 256 * 128 * 2.4e9 / 1e12          # 78.64
OPS_PER_CELL = 3
# Per accumulation mode: VALU lane-operations of the recurrence per admissible
# cell and the peak they run against.
#   plain: v_sub, v_min3, v_fma (the square fused into the add)
#   kahan: sub, min3, three compares, three selects and a max3 picking the
#          carried compensation (the largest among tied sums), then Kahan's
#          add: fma (square minus compensation), add, sub, sub  (13)
#   fp64:  sub, mul, min, min, add in FP64 (5), against the FP64 vector peak
#          78.6 TFLOP/s = 39.32 T lane-ops/s (an FMA counted as one op)
PEAK_FP64_LANE_OPS_T = 78.6 / 2
#   auto, rebased: the plain cell (the rebased form adds per lane a subtract per
#          received value and a renormalisation every 16-32 steps, ~1-3%, not
#          counted as algorithmic work)
MODE_OPS = {"plain": (3, PEAK_LANE_OPS_T, "TOP/s (FP32 VALU lane-ops)"),
            "auto": (3, PEAK_LANE_OPS_T, "TOP/s (FP32 VALU lane-ops)"),
            "rebased": (3, PEAK_LANE_OPS_T, "TOP/s (FP32 VALU lane-ops)"),
            "kahan": (13, PEAK_LANE_OPS_T, "TOP/s (FP32 VALU lane-ops)"),
            "fp64": (5, PEAK_FP64_LANE_OPS_T, "TOP/s (FP64 VALU lane-ops)")}
# profile summary (profiles/<label>*.md) holding the counter-based HBM traffic of a workload's DP kernel
PROFILE_LABELS = {("c2", "auto", "auto", "f32"): "lane_band_W103_c2",
                  ("c5", "auto", "auto", "f32"): "lane_band_W51_c5",
                  ("c3", "auto", "auto", "f32"): "strip_f64_H16x4_c3",
                  ("c4", "auto", "auto", "f32"): "batched_c4",
                  ("c2m", "auto", "auto", "f32"): "lane_split_P12_c2m"}

WORKLOADS = {
    "c2": "equal-length banded matrix: 1000 random walks x 512, window 51",
    "c5": "many short series: 8000 x 256, window 25",
    "c3": "long series: 500 x 4096, no window",
    "c1": "smallest: 20 x 64, no window",
    "c4": "batched uneven: 64 datasets, N in 10..400, lengths in 64..2048, mixed windows, one plan",
    "c2m": "k-medoids assignment step on the 1000 x 512, window 51 data: every series against 10 medoids "
           "(10,000 listed pairs, dtw_plan_create_pairs)",
}
MEDOIDS = 10


def medoid_pairs(N, k, seed=230704906):
    """Every series against k seeded medoids, as listed (series, medoid) pairs."""
    med = np.sort(np.random.default_rng(seed).choice(N, size=k, replace=False))
    return np.array([[i, m] for m in med for i in range(N)], dtype=np.int32)


def make_datasets(name, dtype="f32", c4_seed=None):
    from paper_2307_04904_amd import synth
    if name == "c4":
        return synth.config4(seed=c4_seed)
    if name == "c3":
        return [synth.config3(dtype=dtype)]
    return [{"c1": synth.config1, "c2": synth.config2, "c2m": synth.config2, "c3": synth.config3,
             "c5": synth.config5}[name]()]


def lane_name(g):
    """Kernel label of a lane-band group of a plan's describe JSON."""
    ppw = g.get("pairs_per_wave", 64)
    return "lane:%d/%s" % (g["W"], g["accum"]) + ("" if ppw == 64 else "/%d-per-wave" % ppw)


def sources_sha256(paths):
    """SHA-256 over the bytes of the given repository files, in order."""
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(kernel_label):
    """HBM bytes per launch recorded in profiles/ for the current kernel sources, else None.

    A profile file lists the sources its kernel is built from ("kernel_sources:
    a b c"), their hash when it was measured ("kernel_source_sha256: ...") and
    the scaled FETCH_SIZE + WRITE_SIZE total ("traffic_bytes_per_launch: ...");
    a change to any of those sources invalidates it.
    """
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", kernel_label + "*.md")):
        fields = {}
        for line in open(path).read().splitlines():
            if ":" in line and line.split(":", 1)[0] in ("kernel_sources", "kernel_source_sha256",
                                                         "traffic_bytes_per_launch"):
                k, v = line.split(":", 1)
                fields[k] = v.strip()
        if len(fields) == 3 and sources_sha256(fields["kernel_sources"].split()) == fields["kernel_source_sha256"]:
            return int(fields["traffic_bytes_per_launch"])
    return None


def cpu_baseline(dsets, gpu_outs, target_s, pair_list=None):
    """Time the FP64 oracle on a seeded sample of pairs (all host cores) and check the GPU on them.

    The sample draws pairs uniformly over all datasets' pairs, puts every
    dataset's series in one buffer and times one threaded oracle call over
    them.  A pilot sample, grown until it takes half a second, sets the size
    of the timed sample to about target_s seconds of oracle work.  With
    pair_list (one dataset), the sample is drawn from the listed pairs and
    gpu_outs[0] is indexed like the list.
    """
    import oracle
    from paper_2307_04904_amd import synth
    rng = np.random.default_rng(12345)
    npairs = np.array([d.n_pairs for d in dsets], dtype=np.int64)

    def sample(k):
        if pair_list is not None:
            idx = rng.integers(0, len(pair_list), size=k)
            return [(0, pair_list[idx, 0].astype(np.int32), pair_list[idx, 1].astype(np.int32), idx)]
        which = rng.choice(len(dsets), size=k, p=npairs / npairs.sum())
        out = []
        for d, ds in enumerate(dsets):
            c = int(np.count_nonzero(which == d))
            if c == 0:
                continue
            i = rng.integers(0, ds.N, size=3 * c + 8)
            j = rng.integers(0, ds.N, size=3 * c + 8)
            keep = i != j
            a = np.minimum(i, j)[keep][:c].astype(np.int32)
            b = np.maximum(i, j)[keep][:c].astype(np.int32)
            N = ds.N
            out.append((d, a, b, a.astype(np.int64) * N - a.astype(np.int64) * (a + 1) // 2 + (b - a - 1)))
        return out

    # every dataset's series in one buffer, so one oracle call spans all sampled pairs
    vals = np.concatenate([synth.stored_as_f64(ds) for ds in dsets])
    base = np.cumsum([0] + [len(ds.values) for ds in dsets])[:-1]
    sbase = np.cumsum([0] + [ds.N for ds in dsets])[:-1]
    offs = np.concatenate([ds.offsets + b for ds, b in zip(dsets, base)])
    lens = np.concatenate([ds.lengths for ds in dsets])

    def run(smp):
        pi = np.concatenate([sbase[d] + a for d, a, _, _ in smp]).astype(np.int32)
        pj = np.concatenate([sbase[d] + b for d, _, b, _ in smp]).astype(np.int32)
        win = np.concatenate([np.full(len(a), dsets[d].window, dtype=np.int32) for d, a, _, _ in smp])
        t0 = time.perf_counter()
        ref, threads = oracle.dtw_pairs(vals, offs, lens, pi, pj, win)
        t = time.perf_counter() - t0
        cells = sum(oracle.band_cells(int(lens[a]), int(lens[b]), int(w_)) for a, b, w_ in zip(pi, pj, win))
        refs, k = [], 0
        for d, a, _, _ in smp:
            refs.append(ref[k:k + len(a)])
            k += len(a)
        return t, refs, cells, threads

    k_cal = 64
    while True:
        t_cal, _, _, _ = run(sample(k_cal))
        if t_cal >= 0.5 or k_cal >= npairs.sum():
            break
        k_cal *= 4
    k = int(min(npairs.sum(), max(k_cal, k_cal * target_s / max(t_cal, 1e-3))))
    smp = sample(k)
    t, refs, c, threads = run(smp)
    rels, zero_bad, n = [], 0, 0
    for (d, pi, pj, kk), ref in zip(smp, refs):
        g = gpu_outs[d][kk].astype(np.float64)
        nz = ref > 0
        rels.append(np.abs(g[nz] - ref[nz]) / ref[nz])
        zero_bad += int(np.count_nonzero(g[~nz] != 0.0))
        n += len(pi)
    rel = np.concatenate(rels) if rels else np.zeros(0)
    return {
        "value": c / t / 1e9, "unit": "GCUPS", "cores": int(threads), "kind": "oracle",
        "sample": "%d seeded random pairs of %s (%.3g admissible cells), FP64, %.1f s" % (
            n, "the listed pairs" if pair_list is not None else "the same workload", c, t),
    }, {"pairs_checked": n, "max_rel_err": float(rel.max()) if rel.size else 0.0,
        "mean_rel_err": float(rel.mean()) if rel.size else 0.0, "zero_mismatch": zero_bad}


def quantisation_error(dsets, dsets_f32, gpu_outs, n_pairs=64):
    """GPU results on 16-bit storage against the FP64 oracle on the FP32 source
    values (reported, not gated): what the 8- or 11-bit input rounding costs."""
    import oracle
    from paper_2307_04904_amd import synth
    ds, src = dsets[0], dsets_f32[0]
    rng = np.random.default_rng(54321)
    i = rng.integers(0, ds.N, size=4 * n_pairs)
    j = rng.integers(0, ds.N, size=4 * n_pairs)
    keep = i != j
    a = np.minimum(i, j)[keep][:n_pairs].astype(np.int32)
    b = np.maximum(i, j)[keep][:n_pairs].astype(np.int32)
    ref, _ = oracle.dtw_pairs(synth.stored_as_f64(src), src.offsets, src.lengths, a, b, src.window)
    k = a.astype(np.int64) * ds.N - a.astype(np.int64) * (a + 1) // 2 + (b - a - 1)
    g = gpu_outs[0][k].astype(np.float64)
    rel = np.abs(g - ref) / ref
    return {"pairs": int(len(a)), "max_rel_err": float(rel.max()), "mean_rel_err": float(rel.mean())}


def make_step(plan, stream, use_graph):
    """One step: an eager plan execute, or the replay of a HIP graph captured from one."""
    if not use_graph:
        return (lambda: plan.execute(stream)), None
    import torch
    plan.execute(stream)  # the first launches load the code objects outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()  # capture needs a stream other than the default one
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            plan.execute(side)
    torch.cuda.synchronize()
    return g.replay, g


def time_steps(step, stream, steps, warmup):
    """(ms per step, wall seconds) over `steps` steps after `warmup`, by events on `stream`."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev0.record(stream)
        for _ in range(steps):
            step()
        ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps, time.perf_counter() - t0


def extra_workloads(dev, stream, steps):
    """Rates of the other workloads in the same run (see the module docstring)."""
    import oracle
    import torch
    from paper_2307_04904_amd import binding, synth
    out = {}

    def rate(dsets, graph, n_steps, accum="auto", autotune=False):
        series = [binding.device_series(ds, dev) for ds in dsets]
        outs = [torch.full((max(1, ds.n_pairs),), float("nan"), device=dev) for ds in dsets]
        t0 = time.perf_counter()
        plan = binding.Plan([(s_, ds.lengths, ds.offsets, ds.window, o) for s_, ds, o in zip(series, dsets, outs)],
                            dtype=dsets[0].dtype, accum=accum, timing=True, autotune=autotune)
        plan_s = time.perf_counter() - t0
        step, g = make_step(plan, stream, graph)
        ms, _ = time_steps(step, stream, n_steps, max(3, n_steps // 10))
        cells = plan.info()["band_cells"]
        kms = []
        for _ in range(5):
            plan.execute(stream)
            kms.append(plan.last_kernel_ms())
        desc = plan.describe()
        del g
        plan.destroy()
        res = {"gcups": round(cells / (ms * 1e-3) / 1e9, 1), "ms_per_step": round(ms, 4),
               "kernel_ms": round(statistics.mean(kms), 4), "band_cells": cells,
               "kernels": sorted({"%s/%s" % (g_["kernel"], g_["accum"]) for g_ in desc["wave_groups"]} |
                                 {lane_name(g_) for g_ in desc["lane_groups"]})}
        if autotune:
            res.update(plan_create_s=round(plan_s, 2), tuned_buckets=len(desc["tuned"]),
                       buckets_switched=sum(1 for b in desc["tuned"] if b["applied"] and b["chosen"] != b["model"]),
                       plan_trials=desc["plan_trials"])
        return res, [o.cpu().numpy() for o in outs]

    c2, _ = rate([synth.config2()], False, max(50, steps // 2))
    out["c2_1000x512_w51"] = dict(c2, description=WORKLOADS["c2"])
    # the k-medoids step on the same data (a pair list; the planner spreads
    # each pair over several lanes), against one pair per lane
    ds2 = synth.config2()
    pairs = medoid_pairs(ds2.N, MEDOIDS)
    series2 = binding.device_series(ds2, dev)
    km = {}
    for ppw in (0, 64):
        o = torch.full((len(pairs),), float("nan"), device=dev)
        plan = binding.PairPlan(series2, ds2.lengths, ds2.offsets, ds2.window, pairs, o, timing=True,
                                pairs_per_wave=ppw)
        step, g = make_step(plan, stream, False)
        ms, _ = time_steps(step, stream, 200, 20)
        kms = []
        for _ in range(5):
            plan.execute(stream)
            kms.append(plan.last_kernel_ms())
        desc = plan.describe()
        del g
        plan.destroy()
        km[ppw] = (ms, statistics.mean(kms), desc["lane_groups"][0]["pairs_per_wave"])
    out["c2m_kmedoids_step"] = {
        "pairs": len(pairs), "ms_per_step": round(km[0][0], 4), "kernel_ms": round(km[0][1], 4),
        "pairs_per_wave": km[0][2], "one_pair_per_lane_ms_per_step": round(km[64][0], 4),
        "one_pair_per_lane_kernel_ms": round(km[64][1], 4), "speedup_kernel": round(km[64][1] / km[0][1], 2),
        "description": WORKLOADS["c2m"]}
    c4, c4_outs = rate(synth.config4(), True, 20)
    c4["ratio_to_equal_size_rate"] = round(c4["gcups"] / c2["gcups"], 4)
    out["c4_batched_64_datasets"] = dict(c4, description=WORKLOADS["c4"], timing="hip graph replays")
    c4t, _ = rate(synth.config4(), True, 20, autotune=True)
    c4t["ratio_to_model_plan"] = round(c4t["gcups"] / c4["gcups"], 4)
    out["c4_batched_autotuned"] = dict(c4t, description=WORKLOADS["c4"] + "; DTW_FLAG_AUTOTUNE (measured "
                                       "instances, whole-plan trials)", timing="hip graph replays")
    ds3 = synth.config3()
    c3, c3_out = rate([ds3], False, 10)
    pi, pj = [], []
    rng = np.random.default_rng(4096)
    while len(pi) < 300:
        i, j = sorted(rng.integers(0, ds3.N, size=2))
        if i != j:
            pi.append(i)
            pj.append(j)
    pi, pj = np.array(pi, dtype=np.int32), np.array(pj, dtype=np.int32)
    ref, _ = oracle.dtw_pairs(synth.stored_as_f64(ds3), ds3.offsets, ds3.lengths, pi, pj, ds3.window)
    k = pi.astype(np.int64) * ds3.N - pi.astype(np.int64) * (pi + 1) // 2 + (pj - pi - 1)
    rel = np.abs(c3_out[0][k].astype(np.float64) - ref) / ref
    c3.update(accum="auto (FP64 sums on these unwindowed 8,191-cell paths)", pairs_checked=len(pi),
              max_rel_err=float(rel.max()), mean_rel_err=float(rel.mean()), description=WORKLOADS["c3"])
    out["c3_500x4096_default_accumulation"] = c3
    # the headline matrix with its series stored as BF16 / FP16 (widened to
    # FP32 once by the staging kernel; error against the oracle on the stored
    # values, whose bound is 1e-3 for these forms)
    ds5 = synth.config5()
    rng = np.random.default_rng(8000)
    a5, b5 = rng.integers(0, ds5.N, size=(2, 6000))
    keep = a5 != b5
    pi5, pj5 = np.minimum(a5, b5)[keep].astype(np.int32), np.maximum(a5, b5)[keep].astype(np.int32)
    k5 = pi5.astype(np.int64) * ds5.N - pi5.astype(np.int64) * (pi5 + 1) // 2 + (pj5 - pi5 - 1)
    for dt in ("bf16", "f16"):
        dsd = synth.with_dtype(ds5, dt)
        r5, o5 = rate([dsd], False, 20)
        ref, _ = oracle.dtw_pairs(synth.stored_as_f64(dsd), dsd.offsets, dsd.lengths, pi5, pj5, dsd.window)
        rel = np.abs(o5[0][k5].astype(np.float64) - ref) / np.maximum(ref, 1e-300)
        r5.update(storage=dt, pairs_checked=int(len(pi5)), max_rel_err=float(rel.max()),
                  mean_rel_err=float(rel.mean()), description=WORKLOADS["c5"] + ", series stored as " + dt)
        out["c5_8000x256_w25_%s_storage" % dt] = r5
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed steps; the first launches after the synchronisation wait ~1.8 ms in all for "
                         "the GPU to pick up work, which 20 steps of c2 would count as 6%% of the time")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--kernel", default="auto", choices=["auto", "lane", "wave", "cyclic"])
    ap.add_argument("--accum", default="auto", choices=["auto", "plain", "rebased", "kahan", "fp64"])
    ap.add_argument("--rows-per-lane", type=int, default=0,
                    help="force the strip / cyclic rows per lane (0 = cost model)")
    ap.add_argument("--pairs-per-wave", type=int, default=0, choices=[0, 2, 4, 5, 8, 16, 64],
                    help="force the lane-band kernel's pairs per wavefront (0 = automatic)")
    ap.add_argument("--silhouette", type=int, default=0, metavar="K",
                    help="also time dtw_silhouette on the computed matrix with K seeded random clusters")
    ap.add_argument("--path", action="store_true",
                    help="also time dtw_path (cost matrix, backtrack, row-major matrix) on series 0 and 1")
    ap.add_argument("--autotune", action="store_true",
                    help="plan with DTW_FLAG_AUTOTUNE (kernel instances measured per length/window bucket)")
    ap.add_argument("--dispatch", default="queue", choices=["queue", "hw"],
                    help="work distribution: resident workgroups pulling from a device queue, or one workgroup per item")
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"],
                    help="storage type of the series (the long-series workload's precision study)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target duration of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--describe", metavar="FILE", default="",
                    help="write the plan's kernel groups (dtw_plan_describe JSON) to FILE")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra workloads of the default run (equal-size, k-medoids list, batched graph, "
                         "long series, BF16/FP16 storage)")
    ap.add_argument("--c4-seed", type=int, default=None,
                    help="with --workload c4: another instance of the batched recipe (a workload the cost model "
                         "was not calibrated on)")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of a HIP graph captured from one execute instead of eager executes")
    ap.add_argument("--copy-calibration-mb", type=float, default=0.0,
                    help="only run 5 device-to-device copies of this many MiB (reference for HBM byte counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only (the all-pairs matrix shards by pair ranges with no exchange "
              "between GPUs, so one GPU's share is the measured unit). Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    from paper_2307_04904_amd import binding

    if args.copy_calibration_mb > 0:
        n = int(args.copy_calibration_mb * 2 ** 20) // 4
        src = torch.rand(n, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": 4 * n, "copies": 5}), flush=True)
        return 0

    dsets = make_datasets(args.workload, args.dtype, args.c4_seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    series = [binding.device_series(ds, dev) for ds in dsets]
    pair_list = medoid_pairs(dsets[0].N, MEDOIDS) if args.workload.endswith("m") else None
    n_out = [len(pair_list)] if pair_list is not None else [ds.n_pairs for ds in dsets]
    outs = [torch.full((max(1, k),), float("nan"), dtype=torch.float32, device=dev) for k in n_out]
    t_plan = time.perf_counter()
    if pair_list is not None:
        plan = binding.PairPlan(series[0], dsets[0].lengths, dsets[0].offsets, dsets[0].window, pair_list, outs[0],
                                dtype=dsets[0].dtype, accum=args.accum, kernel=args.kernel, timing=True,
                                queue=args.dispatch == "queue", autotune=args.autotune,
                                pairs_per_wave=args.pairs_per_wave)
    else:
        plan = binding.Plan([(s_, ds.lengths, ds.offsets, ds.window, o) for s_, ds, o in zip(series, dsets, outs)],
                            dtype=dsets[0].dtype, accum=args.accum, kernel=args.kernel, timing=True,
                            queue=args.dispatch == "queue", autotune=args.autotune,
                            rows_per_lane=args.rows_per_lane, pairs_per_wave=args.pairs_per_wave)
    plan_s = time.perf_counter() - t_plan
    info = plan.info()
    plan_desc = plan.describe()
    if args.describe:
        with open(args.describe, "w") as f:
            json.dump(plan_desc, f)
    stream = torch.cuda.current_stream(dev)

    step, graph = make_step(plan, stream, args.graph)
    ms_per_step, wall = time_steps(step, stream, args.steps, args.warmup)

    # DP-kernel-only durations (HIP events recorded by the library on the same stream)
    kms = []
    for _ in range(max(3, min(args.steps, 20))):
        plan.execute(stream)
        kms.append(plan.last_kernel_ms())
    k_avg = statistics.mean(kms)

    cells = info["band_cells"]
    value = cells / (ms_per_step * 1e-3) / 1e9
    # the roofline of the accumulation the plan actually runs (AUTO resolves per pair:
    # all-FP64 plans against the FP64 peak, otherwise the FP32 cell)
    accs = {g["accum"] for g in plan_desc["wave_groups"]} | {g["accum"] for g in plan_desc["lane_groups"]}
    mode = args.accum
    if mode == "auto":
        mode = "fp64" if accs == {"fp64"} else ("kahan" if accs == {"kahan"} else "auto")
    ops_cell, peak, peak_unit = MODE_OPS[mode]
    achieved = ops_cell * cells / (k_avg * 1e-3) / 1e12
    line = {
        "metric": "DTW cell updates/s (GCUPS) for all-pairs matrix; % of FP32 VALU peak",
        "value": round(value, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if mode == "fp64" else "f32",
        "data": "synthetic",
        "timing": "hip graph replays" if args.graph else "eager executes",
        "config": {"workload": (dsets[0].name + ("_medoids%d" % MEDOIDS if pair_list is not None else "")
                                if len(dsets) == 1 else args.workload + "_batched_64_datasets"
                                + ("" if args.c4_seed is None else "_seed%d" % args.c4_seed)),
                   "description": WORKLOADS[args.workload], "datasets": len(dsets),
                   "N": [ds.N for ds in dsets] if len(dsets) > 1 else dsets[0].N,
                   "length": int(max(ds.lengths.max() for ds in dsets)),
                   "window": [ds.window for ds in dsets] if len(dsets) > 1 else dsets[0].window,
                   "pairs": info["pairs"], "band_cells": cells, "swept_cells": info["computed_cells"],
                   "kernel": args.kernel, "accum": args.accum, "accum_groups": sorted(accs),
                   "storage": dsets[0].dtype,
                   "dispatch": args.dispatch, "autotune": args.autotune, "rows_per_lane": args.rows_per_lane,
                   "pairs_per_wave": args.pairs_per_wave,
                   "kernels": ["%s/%s" % (g["kernel"], g["accum"]) for g in plan_desc["wave_groups"]] +
                              [lane_name(g) for g in plan_desc["lane_groups"]],
                   "plan_create_s": round(plan_s, 3), "tuned_buckets": info["n_tuned_buckets"],
                   "tuned_changed": info["n_tuned_changed"]},
        "pct_peak_cell_rate": round(100.0 * value / (PEAK_LANE_OPS_T * 1e3 / OPS_PER_CELL), 2),
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(peak, 2),
            "unit": peak_unit,
            "frac": round(achieved / peak, 4),
            "kernel_ms": round(k_avg, 4),
            "ops_per_cell": ops_cell,
            "ops_per_launch": ops_cell * cells,
            # the profiles were taken with the automatic plan: no traffic for forced shapes or dispatch
            "traffic": recorded_traffic(PROFILE_LABELS.get((args.workload, args.kernel, args.accum, args.dtype), "-"))
            if (args.pairs_per_wave == 0 and args.rows_per_lane == 0 and args.dispatch == "queue"
                and not args.autotune and args.c4_seed is None) else None,
        },
        "wall_s": round(wall, 3),
    }
    if args.silhouette and len(dsets) == 1 and pair_list is None:
        N, K = dsets[0].N, args.silhouette
        labels = torch.from_numpy(np.random.default_rng(7).integers(0, K, size=N).astype(np.int32)).to(dev)
        walls = []
        for _ in range(5):
            t0 = time.perf_counter()
            mean = binding.silhouette(outs[0], N, labels, K, stream=stream)
            walls.append(time.perf_counter() - t0)
        line["silhouette"] = {"K": K, "mean": mean, "call_ms_min": round(1e3 * min(walls), 3),
                              "matrix_bytes": 4 * N * (N - 1) // 2}
    if args.path and dsets[0].dtype == "f32":
        ds = dsets[0]
        o0, o1 = int(ds.offsets[0]), int(ds.offsets[1])
        n, m = int(ds.lengths[0]), int(ds.lengths[1])
        x = series[0][o0:o0 + n].float().contiguous()
        y = series[0][o1:o1 + m].float().contiguous()
        buf = torch.empty(2 * (n + m - 1), dtype=torch.int32, device=dev)
        Cm = torch.empty(n * m, dtype=torch.float32, device=dev)
        res = {}
        for tag, C_out in (("path", None), ("path_and_matrix", Cm)):
            walls = []
            for _ in range(5):
                t0 = time.perf_counter()
                p, cost = binding.warping_path(x, y, ds.window, path_out=buf, C_out=C_out, stream=stream)
                walls.append(time.perf_counter() - t0)
            res[tag + "_call_ms_min"] = round(1e3 * min(walls), 3)
        line["path"] = dict(n=n, m=m, window=ds.window, cells=n * m, path_cells=int(p.shape[0]), cost=cost, **res)
    if not args.no_cpu_baseline:
        torch.cuda.synchronize(dev)
        base, check = cpu_baseline(dsets, [o.cpu().numpy() for o in outs], args.cpu_seconds, pair_list)
        line["cpu_baseline"] = base
        line["gpu_vs_oracle_on_sample"] = check
        if dsets[0].dtype != "f32" and len(dsets) == 1:
            line["gpu_vs_oracle_on_fp32_source"] = quantisation_error(
                dsets, make_datasets(args.workload, "f32"), [o.cpu().numpy() for o in outs])
    del graph  # the captured graph refers to the plan's workspace
    plan.destroy()
    if args.workload == "c5" and not args.no_extra and pair_list is None and args.accum == "auto" \
            and args.kernel == "auto" and args.dtype == "f32":
        line["extra"] = extra_workloads(dev, stream, args.steps)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
