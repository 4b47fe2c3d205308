#!/usr/bin/env python3
"""Throughput of the accelerated-expression hot path on one MI355X.

Default workload ("nested"): the nested map(reduce) configuration, forward and
backward, on seeded synthetic data resident in HBM:
  1. marshaling (device part): row lengths -> offsets (exclusive scan)
  2. ragged row sums, map (reduce (+) 0) over 65536 float32 rows with lengths
     log-uniform in [1, 4096]
  3. dense nested map-map-reduce C = A B, 2048 x 2048 x 2048 FP32 (matrix cores)
  4. reverse of 2: broadcast of the row gradients over the rows
  5. reverse of 3: dA = dC B^T and dB = A^T dC
One "step" is the whole sequence.  `value` counts elements per second, where an
element is one application of the innermost map2 / reduce body: one add per
ragged value (forward), one write per value (reverse), one multiply-add per
(i, j, k) of each of the three matrix products.

The default line also carries `hbm` (the ragged half of the step alone, cold,
against 8 TB/s and against the measured read-only ceiling) and `suite`: the
fused dot, the N-body loop, k-means and the batched expressions, each with its
plain comparison and the roofline of its dominant kernel (--no-suite skips
them).

Other workloads (--workload): dot (fused map2+reduce vs plain), nbody, kmeans,
batched, expr (a user-defined map body, fused map+reduce and reverse mode vs
the same body from the fixed operators), parboil (histogram, stencil, mri-q).
Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "elem/s & HBM GB/s (frac of peak), fused map/reduce fwd+bwd vs plain"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X FP32 vector


# HBM bytes per launch of each roofline kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by the ratio of
# known bytes to counted bytes for the copy kernel (bench.py --copy-calibration).
# `source` is the SHA-256 of the kernel's source file when the counters were
# taken: once that file changes the figure no longer describes the kernel and
# the bench reports null.
TRAFFIC = {
    # k_gemm_mfma<128,128,4,4,TA,TB>, 2048^3, each transpose: 100.77 MB fetched + 16.78 MB written.
    # Each XCD's L2 fetches the A row panels and B column panels of its own 32 tiles (4 x 8 of them:
    # 12 panels of 1 MiB, the fewest 32 tiles can need), so each A panel is fetched by two XCDs and
    # each B panel by four; the algorithmic minimum is 33.6 MB read + 16.8 MB written (2.34x)
    "gemm_nn": {"file": "gemm.hip", "bytes": 117556154,
                "source": "3fa3f9cc142e6e3fc95d3119b28c30c57cd618a098fbb99592d7b86d88652302"},
    "gemm_nt": {"file": "gemm.hip", "bytes": 117533627,
                "source": "3fa3f9cc142e6e3fc95d3119b28c30c57cd618a098fbb99592d7b86d88652302"},
    "gemm_tn": {"file": "gemm.hip", "bytes": 117545915,
                "source": "3fa3f9cc142e6e3fc95d3119b28c30c57cd618a098fbb99592d7b86d88652302"},
    # k_seg_span (row-span path, nontemporal loads), 65536 rows / 32.1 M values: 132.97 MB fetched + 0.26 MB
    # written (1.03x algorithmic: 129.19 MB)
    "seg_span": {"file": "segmented.hip", "bytes": 133236853,
                 "source": "a8bece18ab4e27185c0dc7f3fd5dd1e17669a291e87375a06719fcbf9360ccc5"},
    # mx_xvjp (generated from expr.hip) for exp(-(a-b)^2)*0.5 + a*b over 2^26 float32 pairs:
    # 536.89 MB fetched + 536.83 MB written (1.00x algorithmic)
    "expr_vjp": {"file": "expr.hip", "bytes": 1073735829,
                 "source": "61460c2f96be411e8917cad03f7a568e43228502abc50e0cff6db2ebedee319d"},
    # mx_xseg_add, same body over the nested step's 65 536 ragged rows (2 x 32.1 M values):
    # 261.14 MB fetched + 0.26 MB written (1.01x algorithmic)
    "expr_seg": {"file": "expr.hip", "bytes": 261411148,
                 "source": "61460c2f96be411e8917cad03f7a568e43228502abc50e0cff6db2ebedee319d"},
    # k_stencil7, 512 x 512 x 64 float32: 73.15 MB fetched (1.09x: a 16-plane slab re-reads the planes
    # below and above it) + 67.10 MB written
    "stencil": {"file": "parboil.hip", "bytes": 140264894,
                "source": "43811f5900aa96af3dc0bca90ae62f896a5a0aac06bc3e30816ec5f7f6f67ece"},
    # k_kmeans_fused<32,64,true>, 2^20 x 32 points, k = 64: 134.68 MB fetched (X, 1.00x) + 12.11 MB written
    # (labels, and 768 block partials stored in 32-byte entry groups)
    "kmeans": {"file": "kmeans.hip", "bytes": 146787426,
               "source": "95677d42d858d4619795cb5ed38f6f76aab63f86eb15388f06b026b39355abe0"},
    # k_seg_broadcast (row-span path): 2.66 MB fetched (offsets, gradients) + 128.71 MB written
    "seg_broadcast": {"file": "segmented.hip", "bytes": 131368857,
                      "source": "a8bece18ab4e27185c0dc7f3fd5dd1e17669a291e87375a06719fcbf9360ccc5"},
}


def traffic_of(key):
    import hashlib
    t = TRAFFIC.get(key)
    if t is None:
        return None
    path = os.path.join(ROOT, "paper_2211_00621_amd", "csrc", t["file"])
    with open(path, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["source"]:
            return None
    return t["bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gbs(nbytes, ms):
    return nbytes / (ms * 1e-3) / 1e9


def timed_on(stream, fn, steps, warmup):
    """Run `warmup` untimed calls, then time exactly `steps` calls of fn on
    `stream` between two HIP events, synchronising before and after; returns
    ms per call."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def per_launch_ms(fn, reps=20, warmup=3):
    """Average duration of one launch: `reps` back-to-back launches of fn on
    the current stream between two events (no marker between launches)."""
    import torch
    return timed_on(torch.cuda.current_stream(), fn, reps, warmup)


def launch_stats(fn, reps=50, warmup=3, stream=None):
    """Per-launch durations in ms: each of `reps` launches of fn between its
    own pair of events on `stream` (the current stream by default).  Returns
    the numpy array of durations."""
    import torch
    stream = torch.cuda.current_stream() if stream is None else stream
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in evs])


def summary_us(t):
    """mean / median / p10 / p90 of per-launch durations (ms in, us out)."""
    t = np.asarray(t) * 1e3
    return {"mean_us": round(float(t.mean()), 2), "median_us": round(float(np.median(t)), 2),
            "p10_us": round(float(np.percentile(t, 10)), 2), "p90_us": round(float(np.percentile(t, 90)), 2),
            "reps": int(t.size)}


def rotating(copies, fn):
    """A launcher that calls fn(copy) over `copies` in turn (more bytes than
    the last-level cache holds, so each launch streams from HBM)."""
    turn = [0]

    def f():
        turn[0] = (turn[0] + 1) % len(copies)
        fn(copies[turn[0]])
    return f


def hbm_read_ceiling(dev, nbytes, reps=50):
    """What the chip streams read-only: mx_stream_read (one contiguous 16 KB
    chunk per block, 16-byte loads, one plain store per block) over four rotating buffers of nbytes
    (cold: 4 x nbytes exceeds the 256 MB last-level cache when nbytes is
    ~129 MB).  Per-launch durations, events around each launch."""
    import torch
    from paper_2211_00621_amd import abi
    n = nbytes // 16 * 4
    bufs = [torch.full((n,), i + 1, dtype=torch.int32, device=dev) for i in range(4)]
    x = torch.zeros(abi.MX_STREAM_READ_SLOTS, dtype=torch.int32, device=dev)
    t = launch_stats(rotating(bufs, lambda b: abi.mx_stream_read(b, x)), reps=reps)
    med = float(np.median(t))
    del bufs
    return {"kernel": "k_stream_read", "bytes": 4 * n, **summary_us(t), "GB/s": round(gbs(4 * n, med), 1),
            "frac_hbm": round(gbs(4 * n, med) / HBM_PEAK_GBS, 4)}


def capture(stream, fn):
    """fn() once eagerly on `stream`, then captured into a HIP graph."""
    import torch
    from paper_2211_00621_amd import abi
    with torch.cuda.stream(stream):
        fn()
        stream.synchronize()
        abi.mx_graph_begin(stream)
        fn()
        g = abi.mx_graph_end(stream)
    stream.synchronize()
    return g


def cpu_threads():
    """Host threads for the oracle's parallel leg: the cores this process may
    run on, at most OMP_NUM_THREADS when that is set (the GPU host's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def split_ranges(n, parts):
    """`parts` contiguous [lo, hi) ranges covering range(n)."""
    b = np.linspace(0, n, parts + 1).astype(np.int64)
    return [(int(b[i]), int(b[i + 1])) for i in range(parts) if b[i + 1] > b[i]]


# ============================================================ nested map(reduce)
NESTED = dict(nseg=65536, lmax=4096, M=2048, N=2048, K=2048, seed=0)


def nested_inputs(dev, cfg=NESTED):
    import torch
    import workloads as W
    L, v = W.ragged_f32(cfg["nseg"], cfg["seed"], cfg["lmax"])
    A, B = W.dense_f32(cfg["M"], cfg["N"], cfg["K"], cfg["seed"])
    rng = np.random.default_rng(cfg["seed"] + 100)
    g_rows = rng.uniform(-1, 1, cfg["nseg"]).astype(np.float32)
    G = rng.uniform(-1, 1, (cfg["M"], cfg["N"])).astype(np.float32)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    return dict(L=L, v=v, A=A, B=B, g_rows=g_rows, G=G, tL=t(L), tv=t(v), tA=t(A), tB=t(B),
                tg=t(g_rows), tG=t(G))


def bench_nested(args):
    import torch
    from paper_2211_00621_amd import abi, api
    dev = torch.device("cuda:0")
    cfg = NESTED
    log("nested: generating inputs")
    d = nested_inputs(dev)
    nseg, M, N, K = cfg["nseg"], cfg["M"], cfg["N"], cfg["K"]
    nval = int(d["L"].sum())
    offsets = torch.empty(nseg + 1, dtype=torch.int64, device=dev)
    rows = torch.empty(nseg, dtype=torch.float32, device=dev)
    gvals = torch.empty(nval, dtype=torch.float32, device=dev)
    C = torch.empty((M, N), dtype=torch.float32, device=dev)
    gA = torch.empty((M, K), dtype=torch.float32, device=dev)
    gB = torch.empty((K, N), dtype=torch.float32, device=dev)
    ws = api.workspace(abi.MX_WS_SCAN, nseg, device=dev)
    wseg = api.workspace(abi.MX_WS_SEGMENTED, nval, device=dev)
    names = ["offsets", "row_sums", "mmr_fwd", "row_sums_adjoint", "mmr_adjoint_A", "mmr_adjoint_B"]

    def make_parts(plain):
        if plain:
            seg = lambda: abi.mx_segmented_reduce_plain(abi.MX_ADD, d["tv"], offsets, 0.0, rows)  # noqa: E731
        else:
            seg = lambda: abi.mx_segmented_reduce(abi.MX_ADD, d["tv"], offsets, 0.0, rows, wseg)  # noqa: E731
        mmr = abi.mx_map_map_reduce_plain_f32 if plain else abi.mx_map_map_reduce_f32
        return [
            lambda: abi.mx_lengths_to_offsets(d["tL"], offsets, ws),
            seg,
            lambda: mmr(0, 0, d["tA"], d["tB"], C),
            lambda: abi.mx_segmented_sum_adjoint_f32(d["tg"], offsets, gvals),
            lambda: mmr(0, 1, d["tG"], d["tB"], gA),
            lambda: mmr(1, 0, d["tA"], d["tG"], gB),
        ]

    fused_parts, plain_parts = make_parts(False), make_parts(True)

    def step():
        for f in fused_parts:
            f()

    # The same step with the ragged half (offsets, row sums, broadcast;
    # HBM-bound) on a second stream beside the three matrix products
    # (MFMA-bound): the halves share no data.  Measured slower than one
    # stream (the products run one 128 x 128 tile per CU, and ragged blocks
    # on the same CUs stretch the tiles they share a CU with), so it is
    # reported beside the step, not as the step.  Default priority on both.
    rag = torch.cuda.Stream()
    ev_fork, ev_join = torch.cuda.Event(), torch.cuda.Event()

    def two_stream_step():
        cur = torch.cuda.current_stream()
        ev_fork.record(cur)
        rag.wait_event(ev_fork)
        abi.mx_lengths_to_offsets(d["tL"], offsets, ws, stream=rag)
        abi.mx_segmented_reduce(abi.MX_ADD, d["tv"], offsets, 0.0, rows, wseg, stream=rag)
        abi.mx_segmented_sum_adjoint_f32(d["tg"], offsets, gvals, stream=rag)
        ev_join.record(rag)
        abi.mx_map_map_reduce_f32(0, 0, d["tA"], d["tB"], C, stream=cur)
        abi.mx_map_map_reduce_f32(0, 1, d["tG"], d["tB"], gA, stream=cur)
        abi.mx_map_map_reduce_f32(1, 0, d["tA"], d["tG"], gB, stream=cur)
        cur.wait_event(ev_join)

    def plain_step():
        for f in plain_parts:
            f()

    log("nested: fused steps")
    ms = timed_on(torch.cuda.current_stream(), step, args.steps, args.warmup)
    two_ms = timed_on(torch.cuda.current_stream(), two_stream_step, args.steps, args.warmup)
    side = torch.cuda.Stream()
    graph = capture(side, step)
    graph_ms = timed_on(side, lambda: graph.launch(side), args.steps, args.warmup)
    log(f"nested: fused {ms:.3f} ms/step (eager), {graph_ms:.3f} ms/step (HIP graph replay), "
        f"{two_ms:.3f} ms/step (ragged half on a second stream)")
    reps = max(50, args.steps)
    # every part: per-launch durations (events around each launch), and the
    # average over back-to-back launches (no marker between them)
    stats = {nm: launch_stats(f, reps=reps) for nm, f in zip(names, fused_parts)}
    b2b = {nm: per_launch_ms(f, reps=reps) for nm, f in zip(names, fused_parts)}
    # cold: the ragged kernels over four copies of their streamed array in turn
    # (4 x 129 MB, more than the 256 MB last-level cache), so every launch
    # reads or writes its values from HBM
    vcopies = [d["tv"]] + [d["tv"].clone() for _ in range(3)]
    gcopies = [gvals] + [torch.empty_like(gvals) for _ in range(3)]
    cold = {
        "row_sums": launch_stats(rotating(vcopies, lambda v: abi.mx_segmented_reduce(abi.MX_ADD, v, offsets, 0.0,
                                                                                      rows, wseg)), reps=reps),
        "row_sums_adjoint": launch_stats(rotating(gcopies, lambda gv: abi.mx_segmented_sum_adjoint_f32(
            d["tg"], offsets, gv)), reps=reps),
    }
    del vcopies, gcopies
    # context: the vendor library's FP32 product of the same shape (torch.matmul
    # on the ROCm BLAS stack), per-launch events as for the parts
    torch.backends.cuda.matmul.allow_tf32 = False
    C_lib = torch.empty_like(C)
    lib_mm = launch_stats(lambda: torch.matmul(d["tA"], d["tB"], out=C_lib), reps=reps)
    del C_lib
    ceiling = hbm_read_ceiling(dev, 4 * nval, reps=reps)
    log(f"nested: read-only ceiling {ceiling['GB/s']} GB/s over {ceiling['bytes'] / 1e6:.1f} MB")
    psteps = max(1, min(args.steps, 3))
    pms = timed_on(torch.cuda.current_stream(), plain_step, psteps, 1)
    pparts = {nm: per_launch_ms(f, reps=1, warmup=0) for nm, f in zip(names, plain_parts)}
    log(f"nested: plain {pms:.3f} ms/step")

    elems = 2 * nval + 3 * M * N * K
    flops = 2.0 * M * N * K
    bytes_ = {
        "offsets": 8 * nseg + 8 * (nseg + 1),
        "row_sums": 4 * nval + 8 * (nseg + 1) + 4 * nseg,
        "row_sums_adjoint": 4 * nval + 8 * (nseg + 1) + 4 * nseg,
    }
    counted = {"row_sums": traffic_of("seg_span"), "row_sums_adjoint": traffic_of("seg_broadcast"),
               "mmr_fwd": traffic_of("gemm_nn"), "mmr_adjoint_A": traffic_of("gemm_nt"),
               "mmr_adjoint_B": traffic_of("gemm_tn")}
    # algorithmic bytes of each product: both operands read once, C written once
    mmr_bytes = 4 * (M * K + K * N + M * N)
    detail = {}
    for n in names:
        mean = float(stats[n].mean())
        e = {**summary_us(stats[n]), "b2b_us": round(b2b[n] * 1e3, 2), "plain_us": round(pparts[n] * 1e3, 2)}
        if counted.get(n):
            e["traffic_bytes"] = counted[n]
            e["traffic_ratio"] = round(counted[n] / bytes_.get(n, mmr_bytes), 3)
        if n in bytes_:
            med = float(np.median(stats[n]))
            e["GB/s"] = round(gbs(bytes_[n], med), 1)
            e["frac_hbm"] = round(gbs(bytes_[n], med) / HBM_PEAK_GBS, 4)
            if n in cold:
                cmed = float(np.median(cold[n]))
                e["cold"] = summary_us(cold[n])
                e["cold_GB/s"] = round(gbs(bytes_[n], cmed), 1)
                e["cold_frac_hbm"] = round(gbs(bytes_[n], cmed) / HBM_PEAK_GBS, 4)
                e["cold_frac_ceiling"] = round(gbs(bytes_[n], cmed) / ceiling["GB/s"], 4)
        else:
            tf = flops / (mean * 1e-3) / 1e12
            e["TFLOP/s"] = round(tf, 2)
            e["frac_mfma"] = round(tf / FP32_MFMA_PEAK_TFLOPS, 4)
        detail[n] = e
    dom = "mmr_fwd"
    ach = flops / (float(stats[dom].mean()) * 1e-3) / 1e12
    hbm_ms = float(np.median(cold["row_sums"]) + np.median(cold["row_sums_adjoint"]))
    line = {
        "metric": METRIC,
        "value": elems / (ms * 1e-3),
        "unit": "elem/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "nested map(reduce) fwd+bwd: ragged row sums over 65536 float32 rows "
                               "(lengths log-uniform [1,4096]) + dense map-map-reduce 2048x2048x2048 FP32",
                   "rows": nseg, "values": nval, "M": M, "N": N, "K": K, "seed": cfg["seed"],
                   "elements_per_step": elems},
        "roofline": {"bound": "mfma", "kernel": "k_gemm_mfma<128,128,4,4,0,0> (dense map-map-reduce forward)",
                     "achieved": round(ach, 2), "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / FP32_MFMA_PEAK_TFLOPS, 4), "traffic": traffic_of("gemm_nn"),
                     "duration": "mean of per-launch event pairs"},
        # the ragged (HBM) half of the step on its own: values read forward and
        # written backward, from HBM (cold), against 8 TB/s and the read ceiling
        "hbm": {"elements": 2 * nval, "cold_ms": round(hbm_ms, 4),
                "elem/s": 2 * nval / (hbm_ms * 1e-3),
                "GB/s": round(gbs(bytes_["row_sums"] + bytes_["row_sums_adjoint"], hbm_ms), 1),
                "frac_hbm": round(gbs(bytes_["row_sums"] + bytes_["row_sums_adjoint"], hbm_ms) / HBM_PEAK_GBS, 4),
                "read_ceiling": ceiling},
        "parts": detail,
        "library_product": {"what": "torch.matmul FP32 2048^3 (ROCm BLAS), context only", **summary_us(lib_mm),
                            "TFLOP/s": round(flops / (float(lib_mm.mean()) * 1e-3) / 1e12, 2)},
        "plain": {"ms_per_step": pms, "value": elems / (pms * 1e-3),
                  "fused_speedup": round(pms / ms, 2), "what": "the six plain kernels on one stream, eager"},
        "graph_ms_per_step": graph_ms,
        "two_streams_ms_per_step": two_ms,
        "timing": "value and ms_per_step: K eager steps between two events on the launch stream "
                  "(graph_ms_per_step: the same step replayed from a HIP graph; two_streams_ms_per_step: the "
                  "ragged half on a second stream beside the products); parts: per-launch event pairs over "
                  ">= 50 launches (mean, median, p10, p90) and the back-to-back average (b2b_us); cold: the "
                  "ragged kernels over four 129 MB copies in turn",
    }
    line["marshal"] = marshal_rates(d, dev)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_nested(d, rows, C, gA, gB, gvals, offsets)
    del graph
    return line


def marshal_rates(d, dev):
    """Host-side marshaling of the 65 536 ragged rows through the C ABI:
    mx_marshal_rows (gather into pinned staging on host threads, one
    host-to-device copy, device lengths -> offsets scan) and mx_unmarshal_rows
    (one device-to-host copy, scatter into the host rows).  PCIe-inclusive
    rates, not part of `value`."""
    import ctypes
    import torch
    from paper_2211_00621_amd import abi, api
    L, v = d["L"], d["v"]
    off = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    nseg, total = len(L), int(off[-1])
    rows_in = [v[off[i]:off[i + 1]] for i in range(nseg)]
    rows_out = [np.empty(int(L[i]), dtype=np.float32) for i in range(nseg)]
    ptr_in = (ctypes.c_void_p * nseg)(*[r.ctypes.data if r.size else None for r in rows_in])
    ptr_out = (ctypes.c_void_p * nseg)(*[r.ctypes.data if r.size else None for r in rows_out])
    lengths = np.ascontiguousarray(L, dtype=np.int64)
    staging = torch.empty(((total * 4 + 255) // 256) * 256 + 8 * nseg, dtype=torch.uint8, pin_memory=True)
    values = torch.empty(total, dtype=torch.float32, device=dev)
    lens_dev = torch.empty(nseg, dtype=torch.int64, device=dev)
    offs_dev = torch.empty(nseg + 1, dtype=torch.int64, device=dev)
    ws = api.workspace(abi.MX_WS_SCAN, nseg, device=dev)
    lib = abi._L()
    st = torch.cuda.current_stream().cuda_stream

    def h2d():
        abi._check(lib.mx_marshal_rows(ptr_in, lengths.ctypes.data, nseg, 4, staging.data_ptr(),
                                       staging.numel(), values.data_ptr(), lens_dev.data_ptr(),
                                       offs_dev.data_ptr(), ws.data_ptr(), ws.numel(), st), "mx_marshal_rows")
        torch.cuda.synchronize()

    def d2h():
        abi._check(lib.mx_unmarshal_rows(values.data_ptr(), off.ctypes.data, nseg, 4, staging.data_ptr(),
                                         staging.numel(), ptr_out, st), "mx_unmarshal_rows")

    out = {}
    for name, fn in (("host_to_device", h2d), ("device_to_host", d2h)):
        fn()
        t0 = time.perf_counter()
        for _ in range(3):
            fn()
        secs = (time.perf_counter() - t0) / 3
        nbytes = total * 4 + (nseg + 1) * 8
        out[name] = {"ms": round(secs * 1e3, 2), "GB/s": round(nbytes / secs / 1e9, 1)}
    assert np.array_equal(offs_dev.cpu().numpy(), off) and all(
        np.array_equal(a, b) for a, b in zip(rows_out[:64], rows_in[:64])), "marshal round trip"
    out["note"] = "65 536 host rows (128 MB) through the C ABI, PCIe-inclusive; not part of value"
    return out


def cpu_baseline_nested(d, rows, C, gA, gB, gvals, offsets):
    """The oracle on a bounded sample of the same workload, timed on the host
    twice: on one thread (the sequential column of the paper's tables), and on
    all the host threads this process may use, splitting only the outer maps
    (row ranges of the ragged rows, row blocks of the products) -- every fold
    stays a sequential left fold, so both legs give the same values."""
    import concurrent.futures as cf
    import torch
    import oracle as O
    torch.cuda.synchronize()
    log("nested: cpu baseline (oracle)")
    L, v, A, B, G, g = d["L"], d["v"], d["A"], d["B"], d["G"], d["g_rows"]
    sample_rows = 256
    off = O.offsets_from_lengths(L)
    n = len(L) + 2 * int(L.sum()) + 3 * sample_rows * d["B"].shape[1] * A.shape[1]
    At = A[:, :sample_rows].T.copy()  # rows of A^T: the sample of dB = A^T dC

    def rows_part(lo, hi):
        o = off[lo:hi + 1] - off[lo]
        vv = v[off[lo]:off[hi]]
        return O.segmented_reduce(O.ADD, 0.0, vv, o), O.segmented_sum_adjoint(g[lo:hi], o)

    def prod_part(lo, hi):
        return O.matmul(A[lo:hi], B), O.matmul(G[lo:hi], B, tb=True), O.matmul(At[lo:hi], G)

    def run(threads):
        t0 = time.perf_counter()
        if threads == 1:
            parts_r = [rows_part(0, len(L))]
            parts_p = [prod_part(0, sample_rows)]
        else:
            with cf.ThreadPoolExecutor(threads) as ex:
                fr = [ex.submit(rows_part, lo, hi) for lo, hi in split_ranges(len(L), 4 * threads)]
                fp = [ex.submit(prod_part, lo, hi) for lo, hi in split_ranges(sample_rows, threads)]
                parts_r = [f.result() for f in fr]
                parts_p = [f.result() for f in fp]
        secs = time.perf_counter() - t0
        R = np.concatenate([p[0] for p in parts_r])
        gv = np.concatenate([p[1] for p in parts_r])
        Cs, gAs, gBs = (np.concatenate([p[k] for p in parts_p]) for k in range(3))
        return secs, R, gv, Cs, gAs, gBs

    secs1, R, gv, Cs, gAs, gBs = run(1)
    nt = cpu_threads()
    secsN, RN, gvN, CN, gAN, gBN = run(nt)
    same = all(np.array_equal(x, y) for x, y in ((R, RN), (gv, gvN), (Cs, CN), (gAs, gAN), (gBs, gBN)))
    # sample parity: the GPU results of the timed run against the oracle's
    ok = bool(np.array_equal(offsets.cpu().numpy(), off)) and same
    S = O.segmented_reduce(O.ADD, 0.0, np.abs(v), off)
    rg = rows.cpu().numpy().astype(np.float64)
    ok &= bool(np.all(np.abs(rg - R) <= 1e-4 * np.maximum(np.abs(R), S / np.sqrt(np.maximum(L, 1)))))
    ok &= bool(np.array_equal(gvals.cpu().numpy(), gv.astype(np.float32)))
    worst = 0.0
    for got, ref in ((C.cpu().numpy()[:sample_rows], Cs), (gA.cpu().numpy()[:sample_rows], gAs),
                     (gB.cpu().numpy()[:sample_rows], gBs)):
        err = np.abs(got - ref) / np.maximum(np.abs(ref), math.sqrt(A.shape[1]) / 4)
        worst = max(worst, float(err.max()))
    ok &= worst <= 1e-4
    sample = (f"all 65536 row sums and their adjoint, plus {sample_rows} rows of C, dA and dB "
              f"(2048-long folds) of the 2048^3 products")
    return {"value": n / secsN, "unit": "elem/s", "cores": nt, "kind": "oracle", "seconds": round(secsN, 2),
            "sample": sample, "cpu": cpu_model(),
            "split": "outer maps only (row ranges, product row blocks); folds sequential",
            "single_thread": {"value": n / secs1, "cores": 1, "seconds": round(secs1, 2)},
            "sample_parity": "ok" if ok else "MISMATCH", "max_rel_err_products": worst}


# ============================================================ dot (fused vs plain)
def bench_dot(args):
    import torch
    import workloads as W
    from paper_2211_00621_amd import abi, api
    dev = torch.device("cuda:0")
    n = 1 << 20
    a, b = W.dot_f32(n, 0)
    ai, bi = W.dot_i32(n, 0)
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    tai, tbi = torch.from_numpy(ai).to(dev), torch.from_numpy(bi).to(dev)
    out = torch.empty((), dtype=torch.float32, device=dev)
    outi = torch.empty((), dtype=torch.int64, device=dev)
    tmp = torch.empty(n, dtype=torch.float32, device=dev)
    ws = api.workspace(abi.MX_WS_REDUCE, n, device=dev)
    parts = {
        "fused_f32": per_launch_ms(lambda: abi.mx_map2_reduce(abi.MX_B_MUL, abi.MX_ADD, ta, tb, 0.0, out, ws),
                                   reps=args.steps, warmup=args.warmup),
        "fused_i32": per_launch_ms(lambda: abi.mx_map2_reduce(abi.MX_B_MUL, abi.MX_ADD, tai, tbi, 0, outi, ws),
                                   reps=args.steps, warmup=args.warmup),
        "plain_map2": per_launch_ms(lambda: abi.mx_map2(abi.MX_B_MUL, ta, tb, tmp), reps=args.steps,
                                    warmup=args.warmup),
        "plain_reduce": per_launch_ms(lambda: abi.mx_reduce(abi.MX_ADD, tmp, 0.0, out, ws), reps=args.steps,
                                      warmup=args.warmup),
    }
    # the same K steps captured in one HIP graph and replayed: a 2^20 dot takes
    # a few microseconds on the GPU, less than issuing it from Python, so the
    # eager figure above measures the host; the replay measures the kernels
    side = torch.cuda.Stream()

    def k_steps():
        for _ in range(args.steps):
            abi.mx_map2_reduce(abi.MX_B_MUL, abi.MX_ADD, ta, tb, 0.0, out, ws)

    for _ in range(args.warmup):
        abi.mx_map2_reduce(abi.MX_B_MUL, abi.MX_ADD, ta, tb, 0.0, out, ws)
    graph = capture(side, k_steps)
    graph.launch(side)
    side.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(side)
    graph.launch(side)
    ev1.record(side)
    side.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    assert abs(float(out.cpu()) - float(np.dot(a.astype(np.float64), b.astype(np.float64)))) <= \
        1e-4 * float(np.dot(np.abs(a).astype(np.float64), np.abs(b).astype(np.float64))), "dot result"
    del graph
    sweep = {}
    for k in (24, 26):
        nn = 1 << k
        x = torch.rand(nn, device=dev)
        y = torch.rand(nn, device=dev)
        us = per_launch_ms(lambda: abi.mx_map2_reduce(abi.MX_B_MUL, abi.MX_ADD, x, y, 0.0, out, ws)) * 1e3
        sweep[f"2^{k}"] = {"us": round(us, 2), "GB/s": round(gbs(8 * nn, us * 1e-3), 1),
                           "frac_hbm": round(gbs(8 * nn, us * 1e-3) / HBM_PEAK_GBS, 4)}
    fused = parts["fused_f32"]
    plain = parts["plain_map2"] + parts["plain_reduce"]
    line = {
        "metric": METRIC, "value": n / (ms * 1e-3), "unit": "elem/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "dot: map2(*)+reduce(+) over two float32 vectors of 2^20 (+ int32 variant)",
                   "n": n},
        "roofline": {"bound": "hbm", "kernel": "k_reduce<F32,ADD,MUL> + k_reduce_finish (one step, graph replay)",
                     "achieved": round(gbs(8 * n, ms), 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs(8 * n, ms) / HBM_PEAK_GBS, 4), "traffic": None},
        "parts": {k: {"us": round(v * 1e3, 2)} for k, v in parts.items()},
        "timing": "value and ms_per_step: K steps captured in one HIP graph, one replay between two events on "
                  "its stream; parts: K eager launches from Python between two events (host-bound at this size)",
        "plain": {"us": round(plain * 1e3, 2), "fused_speedup": round(plain / fused, 2)},
        "sweep": sweep,
    }
    if not args.no_cpu_baseline:
        import oracle as O
        log("dot: cpu baseline (oracle)")
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 2.0:
            O.dot(a, b)
            reps += 1
        secs = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": reps * n / secs, "unit": "elem/s", "cores": 1,
                                "kind": "oracle", "seconds": round(secs, 2),
                                "sample": f"the float32 dot over 2^20, {reps} times"}
    return line


# ============================================================ N-body loop
# VALU instructions per pair interaction in the inner loop of the fused forward
# pair kernel (gfx950 ISA of k_pairs<STEP>): 3 sub, 3 mul/fma for |d|^2 plus
# eps2, 2 mul for the cube, 1 mul by the mass, 3 fma into the sums = 12, plus
# the v_rsq_f32 on the transcendental unit.
NBODY_VALU_PER_PAIR = 12
# The ALU peak in lane operations per second: the chip's FP32 vector peak,
# 157.3 TFLOP/s = 256 CUs x 4 SIMDs x 32 FMA lanes per clock x 2 flops x
# 2.4 GHz, counts 32 lane operations per clock per SIMD.  (Sixteen, the width
# of one SIMD's non-packed FP32 lanes, is not the limit: the SQ counters of
# k_mriq show 20.1 VALU lane operations per clock per SIMD, 373.5 M wave
# instructions x 64 lanes in 1.163 M cycles of the 2.2 GHz clock over 1024
# SIMDs.)
LANE_OPS_PER_S = 256 * 4 * 32 * 2.4e9


def nbody_peak_pairs_per_s(valu):
    return LANE_OPS_PER_S / valu


def bench_nbody(args):
    import torch
    import workloads as W
    from paper_2211_00621_amd import abi, api
    dev = torch.device("cuda:0")
    n, T, K, eps2, G, dt = 16384, 20, 5, 1e-6, 1.0, 1e-4
    pos, m, vel = W.nbody(n, 0)
    p4 = torch.zeros((n, 4), device=dev)
    p4[:, :3] = torch.from_numpy(pos).to(dev)
    p4[:, 3] = torch.from_numpy(m).to(dev)
    v4 = torch.zeros((n, 4), device=dev)
    ke = torch.empty((), device=dev)
    gx, gv = torch.empty_like(p4), torch.empty_like(p4)
    ws = torch.zeros(abi.mx_nbody_workspace_bytes(n, T, K), dtype=torch.uint8, device=dev)
    pws = torch.zeros(abi.mx_nbody_pair_workspace_bytes(n), dtype=torch.uint8, device=dev)
    xa, va, xb, vb = (torch.zeros_like(p4) for _ in range(4))
    acc = torch.empty_like(p4)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    # graph of the whole loop and its checkpointed reverse
    with torch.cuda.stream(side):
        abi.mx_nbody_ke_grad_f32(p4, v4, eps2, G, dt, T, K, ke, gx, gv, ws, stream=side)  # warm
        side.synchronize()
        abi.mx_graph_begin(side)
        abi.mx_nbody_ke_grad_f32(p4, v4, eps2, G, dt, T, K, ke, gx, gv, ws, stream=side)
        g_full = abi.mx_graph_end(side)
        abi.mx_graph_begin(side)
        for t in range(T):
            src = (p4, v4) if t == 0 else ((xa, va) if t % 2 else (xb, vb))
            dst = (xb, vb) if t % 2 else (xa, va)
            abi.mx_nbody_step_f32(*src, eps2, G, dt, *dst, pws, stream=side)
        g_fwd = abi.mx_graph_end(side)
    side.synchronize()

    def run_graph(g, pt):
        g.launch(side)

    def timed_on(stream, fn, steps, warmup):
        for _ in range(warmup):
            fn(None)
        stream.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn(None)
        b.record(stream)
        stream.synchronize()
        return a.elapsed_time(b) / steps

    log("nbody: graph-captured loop + checkpointed reverse")
    ms = timed_on(side, lambda pt: run_graph(g_full, pt), args.steps, args.warmup)
    ms_fwd = timed_on(side, lambda pt: run_graph(g_fwd, pt), args.steps, args.warmup)
    log(f"nbody: fwd+bwd {ms:.3f} ms, fwd {ms_fwd:.3f} ms")

    # per-launch durations of the pair kernels (eager, events on the launch stream)
    parts = {"step": per_launch_ms(lambda: abi.mx_nbody_step_f32(p4, v4, eps2, G, dt, xa, va, pws), reps=10),
             "adjoint_step": per_launch_ms(
                 lambda: abi.mx_nbody_adjoint_step_f32(p4, xb, va, eps2, G, dt, gx, gv, pws), reps=10)}

    # plain: eager untiled pair loop + separate update, forward only
    def plain_fwd(pt):
        x, v = p4, v4
        for t in range(T):
            dst = (xb, vb) if t % 2 else (xa, va)
            abi.mx_nbody_step_plain_f32(x, v, eps2, G, dt, acc, *dst)
            x, v = dst
    pms = timed_on(torch.cuda.current_stream(), plain_fwd, max(1, min(args.steps, 3)), 1)
    log(f"nbody: plain fwd {pms:.3f} ms")

    pairs_fwd = T * n * n
    pairs_bwd = (T - T // K) * n * n + T * n * n  # recomputed steps + adjoint steps
    peak = nbody_peak_pairs_per_s(NBODY_VALU_PER_PAIR)
    ach = n * n / (parts["step"] * 1e-3)
    line = {
        "metric": METRIC, "value": (pairs_fwd + pairs_bwd) / (ms * 1e-3), "unit": "pair-interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "loop around pairwise map(reduce): N-body N=16384, 20 Euler steps, dt=1e-4, "
                               "eps=1e-3, fwd + adjoint of final KE wrt x0 with checkpoints every 5 steps",
                   "n": n, "steps": T, "ckpt_every": K},
        "roofline": {"bound": "alu", "kernel": "k_pairs<STEP> (+ slice finish)",
                     "achieved": round(ach / 1e9, 1), "peak": round(peak / 1e9, 1), "unit": "Gpair/s",
                     "frac": round(ach / peak, 4), "traffic": None,
                     "peak_basis": f"FP32 vector peak as lane operations (256 CU x 4 SIMD x 32 lanes x 2.4 GHz) / "
                                   f"{NBODY_VALU_PER_PAIR} VALU instructions per pair (reciprocal square root on "
                                   "the transcendental unit)"},
        "parts": {"fwd_20_steps_ms": round(ms_fwd, 3), "reverse_ms": round(ms - ms_fwd, 3),
                  "step_launch_us": round(parts["step"] * 1e3, 1),
                  "adjoint_step_launch_us": round(parts["adjoint_step"] * 1e3, 1)},
        "plain": {"fwd_20_steps_ms": round(pms, 3), "fused_speedup_fwd": round(pms / ms_fwd, 2)},
    }
    if not args.no_cpu_baseline:
        import oracle as O
        log("nbody: cpu baseline (oracle)")
        x0 = pos.astype(np.float64)
        t0 = time.perf_counter()
        O.nbody_step(x0, vel, m, eps2, G, dt)
        O.nbody_accel_vjp(x0, m, np.ones_like(x0), eps2, G)
        secs = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 2 * n * n / secs, "unit": "pair-interactions/s", "cores": 1,
                                "kind": "oracle", "seconds": round(secs, 2),
                                "sample": "one forward Euler step and one transposed-Jacobian product at N=16384"}
    del g_full, g_fwd
    return line


# ============================================================ k-means
def bench_kmeans(args):
    import torch
    import workloads as W
    from paper_2211_00621_amd import abi, api
    dev = torch.device("cuda:0")
    n, d, k, iters = 1 << 20, 32, 64, 10
    X, _, _ = W.kmeans_blobs(n, d, k, seed=0)
    Xt = torch.from_numpy(X).to(dev)
    Cs = [Xt[:k].clone()] + [torch.empty((k, d), device=dev) for _ in range(iters)]
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    counts = torch.empty(k, dtype=torch.int64, device=dev)
    ws = torch.zeros(abi.mx_kmeans_workspace_bytes(n, d, k), dtype=torch.uint8, device=dev)
    sse = torch.empty((), device=dev)
    sse_ws = torch.zeros(256 + 4096, dtype=torch.uint8, device=dev)
    one = torch.ones(1, device=dev)
    G = torch.empty_like(Xt)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()

    def body(step_fn, stream):
        for it in range(iters):
            step_fn(Xt, Cs[it], labels, counts, Cs[it + 1], ws, stream=stream)
        abi.mx_kmeans_sse_f32(Xt, Cs[iters], labels, sse, sse_ws, stream=stream)
        abi.mx_kmeans_sse_grad_f32(Xt, Cs[iters], labels, one, G, stream=stream)

    with torch.cuda.stream(side):
        body(abi.mx_kmeans_step_f32, side)
        side.synchronize()
        abi.mx_graph_begin(side)
        body(abi.mx_kmeans_step_f32, side)
        graph = abi.mx_graph_end(side)
    side.synchronize()

    ms = timed_on(side, lambda: graph.launch(side), args.steps, args.warmup)
    cur = torch.cuda.current_stream()
    pms = timed_on(cur, lambda: body(abi.mx_kmeans_step_plain_f32, None), max(1, min(args.steps, 5)), 1)

    parts = {"kmeans_step": per_launch_ms(lambda: abi.mx_kmeans_step_f32(Xt, Cs[0], labels, counts, Cs[1], ws)),
             "sse_grad": per_launch_ms(lambda: abi.mx_kmeans_sse_grad_f32(Xt, Cs[1], labels, one, G))}
    log(f"kmeans: fused {ms:.3f} ms, plain {pms:.3f} ms")
    flops_step = 2.0 * n * k * d
    ach = flops_step / (parts["kmeans_step"] * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": iters * n * k / (ms * 1e-3), "unit": "point-centroid evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "k-means: 2^20 float32 points in d=32 from 64 Gaussian blobs, k=64, 10 steps of "
                               "map(argmin reduce)+reduce-by-key, then SSE and its gradient wrt the points",
                   "n": n, "d": d, "k": k, "iterations": iters},
        # the step's x.c products run as three bfloat16 products each (high and
        # middle parts), 3 x 2nkd flops at 2.5 PFLOP/s: 5 us, below the 17 us
        # its 138 MB of HBM traffic need at 8 TB/s, so HBM is the roofline
        "roofline": {"bound": "hbm", "kernel": "k_kmeans_fused<32,64>",
                     "achieved": round(gbs(4 * n * d + 4 * n, parts["kmeans_step"]), 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs(4 * n * d + 4 * n, parts["kmeans_step"]) / HBM_PEAK_GBS, 4),
                     "traffic": traffic_of("kmeans"),
                     "limit": "VALU issue: ~1100 vector instructions per 64-point chunk (bfloat16 split, "
                              "candidate selection, certification, reduce-by-key), three waves per SIMD",
                     "fp32_equivalent": {"TFLOP/s": round(ach, 2), "of_fp32_mfma_peak": round(ach / FP32_MFMA_PEAK_TFLOPS, 4),
                                         "what": "2nkd flops of the x.c products over the step's time, against the "
                                                 "FP32 matrix peak (the former FP32 16x16x4 kernel's bound)"}},
        "parts": {"kmeans_step_us": round(parts["kmeans_step"] * 1e3, 1),
                  "kmeans_step_GB/s": round(gbs(4 * n * d + 4 * n, parts["kmeans_step"]), 1),
                  "sse_grad_us": round(parts["sse_grad"] * 1e3, 1),
                  "sse_grad_GB/s": round(gbs(8 * n * d + 4 * n, parts["sse_grad"]), 1)},
        "plain": {"ms_per_step": round(pms, 3), "fused_speedup": round(pms / ms, 2)},
    }
    if not args.no_cpu_baseline:
        import oracle as O
        log("kmeans: cpu baseline (oracle)")
        Co = X[:k].astype(np.float64)
        t0 = time.perf_counter()
        for _ in range(iters):
            lab = O.kmeans_assign(X, Co)
            _, _, Co = O.kmeans_update(X, lab, Co)
        secs = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": iters * n * k / secs, "unit": "point-centroid evals/s",
                                "cores": 1, "kind": "oracle", "seconds": round(secs, 2),
                                "sample": f"the whole workload: {iters} assignment + update steps over all "
                                          f"2^20 points (no SSE / gradient)"}
    del graph
    return line


# ============================================================ batched uneven expressions
def bench_batched(args):
    import tempfile
    import torch
    import workloads as W
    from paper_2211_00621_amd import abi, api
    dev = torch.device("cuda:0")
    bt = W.batched_tasks(2048, seed=0)
    tb = bt.table()
    A = torch.from_numpy(bt.A).to(dev)
    B = torch.from_numpy(bt.B).to(dev)
    g = torch.from_numpy(bt.gout).to(dev)
    out = torch.empty(bt.out_len, device=dev)
    gA = torch.empty_like(A)
    gB = torch.empty_like(B)
    batch = api.Batch(tb, device=dev)
    cache = os.environ.get("MX_TUNE_CACHE") or os.path.join(tempfile.gettempdir(), "mx_batch_tune.jsonl")
    log("batched: autotune")
    chosen = batch.autotune(A, B, out, g, gA, gB, cache_path=cache)
    log(f"batched: chosen tile_elems={chosen[0]} blocks_per_cu={chosen[1]}")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        batch.forward(A, B, out, stream=side)
        batch.backward(A, B, g, gA, gB, stream=side)
        side.synchronize()
        abi.mx_graph_begin(side)
        batch.forward(A, B, out, stream=side)
        batch.backward(A, B, g, gA, gB, stream=side)
        graph = abi.mx_graph_end(side)
    side.synchronize()

    ms = timed_on(side, lambda: graph.launch(side), args.steps, args.warmup)
    cur = torch.cuda.current_stream()

    def plain():
        batch.forward(A, B, out, plain=True)
        batch.backward(A, B, g, gA, gB, plain=True)
    pms = timed_on(cur, plain, max(1, min(args.steps, 5)), 1)

    parts = {"forward": per_launch_ms(lambda: batch.forward(A, B, out)),
             "backward": per_launch_ms(lambda: batch.backward(A, B, g, gA, gB))}
    log(f"batched: graph {ms:.3f} ms, plain {pms:.3f} ms")

    rows, cols, kind = bt.rows, bt.cols, bt.kind
    elems = int((rows * cols).sum())
    dot = kind == W.TASK_DOT
    fwd_bytes = int((8 * cols[dot]).sum() + (4 * rows[~dot] * cols[~dot] + 4 * cols[~dot] + 4 * rows[~dot]).sum())
    bwd_bytes = int((16 * cols[dot] + 4).sum()
                    + (8 * rows[~dot] * cols[~dot] + 8 * cols[~dot] + 4 * rows[~dot]).sum())
    ach = gbs(bwd_bytes, parts["backward"])
    line = {
        "metric": METRIC, "value": 2 * elems / (ms * 1e-3), "unit": "elem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched uneven: 2048 dot/matvec expressions, sizes log-uniform 1e2..1e6, "
                               "forward + backward, autotuned persistent launches in a HIP graph",
                   "tasks": 2048, "elements": elems, "tile_elems": chosen[0], "blocks_per_cu": chosen[1]},
        "roofline": {"bound": "hbm", "kernel": "k_batch_bwd (+ combine)", "achieved": round(ach, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None},
        "parts": {"forward_us": round(parts["forward"] * 1e3, 1),
                  "forward_GB/s": round(gbs(fwd_bytes, parts["forward"]), 1),
                  "backward_us": round(parts["backward"] * 1e3, 1), "backward_GB/s": round(ach, 1)},
        "plain": {"ms_per_step": round(pms, 3), "batched_speedup": round(pms / ms, 2)},
    }
    if not args.no_cpu_baseline:
        import oracle as O
        log("batched: cpu baseline (oracle)")
        sample = 2048
        t0 = time.perf_counter()
        O.batch_forward(tb[:sample], bt.A, bt.B, bt.out_len)
        O.batch_backward(tb[:sample], bt.A, bt.B, bt.gout)
        secs = time.perf_counter() - t0
        se = int((rows[:sample] * cols[:sample]).sum())
        line["cpu_baseline"] = {"value": 2 * se / secs, "unit": "elem/s", "cores": 1, "kind": "oracle",
                                "seconds": round(secs, 2),
                                "sample": "forward + backward of all 2048 tasks"}
    del graph
    return line


# ============================================================ user-defined map bodies
def gauss_dot_body(abi):
    """exp(-(a - b)^2) * 0.5 + a * b as a straight-line register program."""
    X = abi
    return [(X.MX_X_IN, 0, 0, 0, 0.0), (X.MX_X_IN, 1, 1, 0, 0.0), (X.MX_X_SUB, 2, 0, 1, 0.0),
            (X.MX_X_SQ, 2, 2, 0, 0.0), (X.MX_X_NEG, 2, 2, 0, 0.0), (X.MX_X_EXP, 2, 2, 0, 0.0),
            (X.MX_X_CONST, 3, 0, 0, 0.5), (X.MX_X_MUL, 2, 2, 3, 0.0), (X.MX_X_MUL, 4, 0, 1, 0.0),
            (X.MX_X_ADD, 2, 2, 4, 0.0)], 2


def bench_expr(args):
    import torch
    from paper_2211_00621_amd import abi, api
    dev = torch.device("cuda:0")
    n = 1 << 26
    gen = torch.Generator(device=dev).manual_seed(0)
    a = torch.rand(n, device=dev, generator=gen) * 2 - 1
    b = torch.rand(n, device=dev, generator=gen) * 2 - 1
    prog, out_reg = gauss_dot_body(abi)
    e = abi.mx_expr_create(prog, 2, out_reg, abi.MX_F32)
    abi.mx_expr_prepare(e)
    ws = torch.zeros(abi.mx_expr_workspace_bytes(e, n), dtype=torch.uint8, device=dev)
    r = torch.empty((), device=dev)
    gs = torch.ones(1, device=dev)
    ga, gb = torch.empty_like(a), torch.empty_like(b)
    t1, t2, t3 = torch.empty_like(a), torch.empty_like(a), torch.empty_like(a)
    red_ws = torch.zeros(abi.mx_workspace_bytes(abi.MX_WS_REDUCE, n, 0), dtype=torch.uint8, device=dev)

    def fwd():
        abi.mx_expr_map_reduce(e, abi.MX_ADD, [a, b], n, 0.0, r, ws)

    def bwd():
        abi.mx_expr_vjp(e, [a, b], n, None, gs, [ga, gb])

    def plain_fwd():  # the same body from the fixed map / map2 bodies, one temporary per step
        abi.mx_map2(abi.MX_B_SUB, a, b, t1)
        abi.mx_map(abi.MX_U_SQ, t1, None, t2)
        abi.mx_map(abi.MX_U_AFFINE, t2, (-1.0, 0.0), t1)
        abi.mx_map(abi.MX_U_EXP, t1, None, t2)
        abi.mx_map(abi.MX_U_AFFINE, t2, (0.5, 0.0), t1)
        abi.mx_map2(abi.MX_B_MUL, a, b, t2)
        abi.mx_map2(abi.MX_B_ADD, t1, t2, t3)
        abi.mx_reduce(abi.MX_ADD, t3, 0.0, r, red_ws)

    parts = {"map_reduce": per_launch_ms(fwd, reps=args.steps, warmup=args.warmup),
             "vjp": per_launch_ms(bwd, reps=args.steps, warmup=args.warmup)}
    # the body inside the nested map(reduce) over the ragged rows of the nested
    # step (65 536 rows, lengths log-uniform [1, 4096]), two value arrays
    import workloads as W
    L = W.ragged_lengths(NESTED["nseg"], NESTED["seed"], NESTED["lmax"])
    off = torch.from_numpy(np.concatenate([[0], np.cumsum(L)]).astype(np.int64)).to(dev)
    nv = int(L.sum())
    va, vb = a[:nv], b[:nv]
    rows = torch.empty(len(L), device=dev)
    tmpv = torch.empty(nv, device=dev)
    wseg = api.workspace(abi.MX_WS_SEGMENTED, nv, device=dev)

    def seg():
        abi.mx_expr_segmented_reduce(e, abi.MX_ADD, [va, vb], off, 0.0, rows)

    def seg_plain():  # body into a temporary, then the fixed ragged row sums
        abi.mx_expr_map(e, [va, vb], tmpv)
        abi.mx_segmented_reduce(abi.MX_ADD, tmpv, off, 0.0, rows, wseg)

    parts["segmented"] = per_launch_ms(seg, reps=args.steps, warmup=args.warmup)
    parts["segmented_plain"] = per_launch_ms(seg_plain, reps=args.steps, warmup=args.warmup)
    seg_bytes = 8 * nv + 8 * (len(L) + 1) + 4 * len(L)
    cur = torch.cuda.current_stream()
    ms = timed_on(cur, lambda: (fwd(), bwd()), args.steps, args.warmup)
    pms = timed_on(cur, plain_fwd, max(1, min(args.steps, 10)), 1)
    fwd_bytes, bwd_bytes = 8 * n, 16 * n
    ach = gbs(bwd_bytes, parts["vjp"])
    log(f"expr: fused fwd {parts['map_reduce'] * 1e3:.1f} us, vjp {parts['vjp'] * 1e3:.1f} us, "
        f"plain fwd {pms * 1e3:.1f} us")
    line = {
        "metric": METRIC, "value": 2 * n / (ms * 1e-3), "unit": "elem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "user-defined map body exp(-(a-b)^2)*0.5 + a*b over two float32 vectors of 2^26: "
                               "fused map+reduce(+) and its reverse mode (runtime-compiled kernels)", "n": n},
        "roofline": {"bound": "hbm", "kernel": "mx_xvjp", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_of("expr_vjp")},
        "parts": {"map_reduce_us": round(parts["map_reduce"] * 1e3, 1),
                  "map_reduce_GB/s": round(gbs(fwd_bytes, parts["map_reduce"]), 1),
                  "vjp_us": round(parts["vjp"] * 1e3, 1), "vjp_GB/s": round(ach, 1),
                  "segmented_rows": len(L), "segmented_values": nv,
                  "segmented_us": round(parts["segmented"] * 1e3, 1),
                  "segmented_GB/s": round(gbs(seg_bytes, parts["segmented"]), 1),
                  "segmented_traffic_bytes": traffic_of("expr_seg"),
                  "segmented_via_temporary_us": round(parts["segmented_plain"] * 1e3, 1)},
        "plain": {"forward_us": round(pms * 1e3, 1), "fused_speedup": round(pms / parts["map_reduce"], 2)},
    }
    if not args.no_cpu_baseline:
        import oracle as O
        log("expr: cpu baseline (oracle)")
        sample = n
        an, bn = a[:sample].cpu().numpy(), b[:sample].cpu().numpy()
        t0 = time.perf_counter()
        O.expr_map_reduce(O.ADD, 0.0, prog, out_reg, an, bn)
        O.expr_vjp(prog, out_reg, [an, bn], gscale=1.0)
        secs = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 2 * sample / secs, "unit": "elem/s", "cores": 1,
                                "kind": "oracle", "seconds": round(secs, 2),
                                "sample": "map+reduce and reverse mode over all 2^26 elements"}
    return line


# ============================================================ Parboil-shaped kernels
# VALU instructions per (voxel, sample) pair in the inner loop of k_mriq
# (gfx950 ISA: 73 per four samples for the thread's two voxels, of which 16
# are v_sin / v_cos on the transcendental unit).
MRIQ_VALU_PER_PAIR = 9.125
# VALU instructions per pair in the inner loop of k_tpacf<32> (gfx950 ISA:
# 89 per four pairs: the dot product, a five-level binary search over the
# edges, two levels from registers and three LDS probes, and the counter
# address); 12 LDS reads and 4 LDS adds per four pairs alongside.
TPACF_VALU_PER_PAIR = 22.25


def bench_parboil(args):
    import torch
    from paper_2211_00621_amd import abi
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(0)
    # histo: 2^24 keys of an image-like (concentrated) distribution
    nkeys = 1 << 24
    keys_np = {nb: np.clip(np.rint(rng.normal(nb * 0.4, nb / 20, nkeys)), 0, nb - 1).astype(np.uint32)
               for nb in (4096, 1 << 20)}
    keys = {nb: torch.from_numpy(k).to(dev).view(torch.int32) for nb, k in keys_np.items()}
    counts = {nb: torch.empty(nb, dtype=torch.int32, device=dev) for nb in keys}
    # stencil: 64 planes of 512 x 512
    nz, ny, nx = 64, 512, 512
    g0 = torch.rand((nz, ny, nx), device=dev) * 2 - 1
    g1 = torch.empty_like(g0)
    # mri-q: 2048 samples, 2^18 voxels
    nk, nv = 2048, 1 << 18
    kxyz = [torch.rand(nk, device=dev) * 32 - 16 for _ in range(3)]
    phi = torch.rand(nk, device=dev)
    xyz = [torch.rand(nv, device=dev) - 0.5 for _ in range(3)]
    qr, qi = torch.empty(nv, device=dev), torch.empty(nv, device=dev)
    # tpacf: 2^15 data and 2^15 random points on the sphere, 20 log-spaced angular edges (0.1 .. 158 deg)
    npt, nedge = 1 << 15, 20
    sph = []
    for sd in (1, 2):
        v = torch.randn((3, npt), device=dev, generator=torch.Generator(device=dev).manual_seed(sd))
        sph.append((v / v.norm(dim=0)).contiguous())
    tp_edges = torch.from_numpy(np.cos(np.radians(np.logspace(-1, 2.2, nedge))).astype(np.float32)).to(dev)
    tp_counts = torch.empty(nedge + 1, dtype=torch.int64, device=dev)

    def tpacf():  # DD (pairs i < j) then DR (all pairs)
        abi.mx_tpacf_f32(sph[0], sph[0], tp_edges, tp_counts, True)
        abi.mx_tpacf_f32(sph[0], sph[1], tp_edges, tp_counts, False)

    def histo_small():
        abi.mx_histogram_u32(keys[4096], 4096, counts[4096])

    hws = torch.zeros(abi.mx_workspace_bytes(abi.MX_WS_HISTOGRAM, nkeys, 1 << 20), dtype=torch.uint8, device=dev)

    def histo_large():  # bucketed: group keys by bucket of 2^11 bins, then LDS counts per bucket
        abi.mx_histogram_u32(keys[1 << 20], 1 << 20, counts[1 << 20], hws)

    def histo_large_atomics():  # the same without a workspace: one global atomic per key
        abi.mx_histogram_u32(keys[1 << 20], 1 << 20, counts[1 << 20])

    def stencil():
        abi.mx_stencil7_f32(g0, g1, 1.0 / 6.0, 0.125)

    def mriq():
        abi.mx_mriq_f32(*kxyz, phi, *xyz, qr, qi)

    def step():
        histo_small()
        histo_large()
        stencil()
        mriq()
        tpacf()

    parts = {nm: per_launch_ms(f, reps=max(args.steps, 5), warmup=args.warmup)
             for nm, f in (("histo_4096_bins", histo_small), ("histo_2^20_bins", histo_large),
                           ("histo_2^20_bins_global_atomics", histo_large_atomics),
                           ("stencil", stencil), ("mriq", mriq), ("tpacf", tpacf))}
    histo_large()
    assert np.array_equal(counts[1 << 20].cpu().numpy().astype(np.int64),
                          np.bincount(keys_np[1 << 20], minlength=1 << 20)), "bucketed histogram"
    ms = timed_on(torch.cuda.current_stream(), step, args.steps, args.warmup)
    pts = nx * ny * nz
    pairs = nk * nv
    tp_pairs = npt * (npt - 1) // 2 + npt * npt
    elems = 2 * nkeys + pts + pairs + tp_pairs
    mriq_peak = LANE_OPS_PER_S / MRIQ_VALU_PER_PAIR
    tp_peak = LANE_OPS_PER_S / TPACF_VALU_PER_PAIR
    tp_rate = tp_pairs / (parts["tpacf"] * 1e-3)
    mriq_rate = pairs / (parts["mriq"] * 1e-3)
    log(f"parboil: step {ms:.3f} ms; " + ", ".join(f"{k} {v * 1e3:.1f} us" for k, v in parts.items()))
    line = {
        "metric": METRIC, "value": elems / (ms * 1e-3), "unit": "elem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "Parboil-shaped kernels on synthetic data: histogram of 2^24 concentrated keys into "
                               "4096 and 2^20 bins, one 7-point stencil sweep of 512x512x64 float32, mri-q with "
                               "2048 samples x 2^18 voxels, tpacf DD + DR pair counts of 2^15 + 2^15 points on "
                               "the sphere in 21 angular bins", "keys": nkeys, "grid": [nz, ny, nx],
                   "mriq": [nk, nv], "tpacf_points": npt, "elements_per_step": elems},
        "roofline": {"bound": "alu", "kernel": "k_tpacf<32>", "achieved": round(tp_rate / 1e9, 1),
                     "peak": round(tp_peak / 1e9, 1), "unit": "Gpair/s", "frac": round(tp_rate / tp_peak, 4),
                     "traffic": None,
                     "peak_basis": f"FP32 vector peak as lane operations (256 CU x 4 SIMD x 32 lanes x 2.4 GHz) / "
                                   f"{TPACF_VALU_PER_PAIR} VALU instructions per pair"},
        "parts": {
            "histo_4096_bins": {"us": round(parts["histo_4096_bins"] * 1e3, 1),
                                "GB/s": round(gbs(4 * nkeys, parts["histo_4096_bins"]), 1)},
            "histo_2^20_bins": {"us": round(parts["histo_2^20_bins"] * 1e3, 1),
                                "GB/s": round(gbs(4 * nkeys, parts["histo_2^20_bins"]), 1)},
            "histo_2^20_bins_global_atomics": {"us": round(parts["histo_2^20_bins_global_atomics"] * 1e3, 1),
                                               "GB/s": round(gbs(4 * nkeys, parts["histo_2^20_bins_global_atomics"]),
                                                             1)},
            "stencil": {"us": round(parts["stencil"] * 1e3, 1), "GB/s": round(gbs(8 * pts, parts["stencil"]), 1),
                        "frac_hbm": round(gbs(8 * pts, parts["stencil"]) / HBM_PEAK_GBS, 4),
                        "traffic_bytes": traffic_of("stencil")},
            "mriq": {"us": round(parts["mriq"] * 1e3, 1), "Gpair/s": round(mriq_rate / 1e9, 1),
                     "frac_alu": round(mriq_rate / mriq_peak, 4),
                     "alu_basis": f"{MRIQ_VALU_PER_PAIR} VALU instructions per pair"},
            "tpacf": {"us": round(parts["tpacf"] * 1e3, 1), "pairs": tp_pairs,
                      "Gpair/s": round(tp_rate / 1e9, 1), "frac_alu": round(tp_rate / tp_peak, 4)},
        },
    }
    if not args.no_cpu_baseline:
        import oracle as O
        log("parboil: cpu baseline (oracle)")
        sample_v, sample_p = 1 << 16, 8192
        g0n = g0.cpu().numpy()
        kn = [t.cpu().numpy() for t in kxyz]
        xn = [t[:sample_v].cpu().numpy() for t in xyz]
        s0, s1 = sph[0].cpu().numpy(), sph[1].cpu().numpy()
        e_np = tp_edges.cpu().numpy()
        t0 = time.perf_counter()
        for nb, k in keys_np.items():
            O.histogram(k, nb)
        O.stencil7(g0n, 1.0 / 6.0, 0.125)
        O.mriq(*kn, phi.cpu().numpy(), *xn)
        O.tpacf(s0[:, :sample_p], s1, e_np, False)
        secs = time.perf_counter() - t0
        n_done = 2 * nkeys + pts + nk * sample_v + sample_p * npt
        line["cpu_baseline"] = {"value": n_done / secs, "unit": "elem/s", "cores": 1, "kind": "oracle",
                                "seconds": round(secs, 2),
                                "sample": f"both histograms and the stencil sweep in full, mri-q for the first "
                                          f"{sample_v} of the 2^18 voxels, tpacf cross pairs of the first {sample_p} "
                                          f"data points with all 2^15 random points"}
    return line


def copy_calibration(mib):
    import torch
    from paper_2211_00621_amd import abi
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        abi.mx_copy32(src, dst)
    torch.cuda.synchronize()
    return {"copy_calibration": {"kernel": "k_copy32", "launches": 5, "read_bytes": n, "write_bytes": n}}


def suite_results(args):
    """The other configurations measured inside the default run, each with its
    own fused and plain forms (fewer timed steps, no CPU baseline): the
    fused dot (2^20), the N-body loop with its checkpointed reverse (16 384
    bodies, 20 steps), k-means (2^20 x 32, k = 64, 10 steps) and the 2048
    batched uneven expressions.  Per workload: value, step time, the roofline
    of its dominant kernel and the plain comparison."""
    import torch
    sub = argparse.Namespace(steps=max(3, min(args.steps, 10)), warmup=2, no_cpu_baseline=True)
    out = {}
    for name, fn in (("dot", bench_dot), ("nbody", bench_nbody), ("kmeans", bench_kmeans),
                     ("batched", bench_batched)):
        t0 = time.perf_counter()
        log(f"suite: {name}")
        ln = fn(sub)
        rf = ln["roofline"]
        out[name] = {"workload": ln["config"]["workload"], "value": ln["value"], "unit": ln["unit"],
                     "ms_per_step": round(ln["ms_per_step"], 4),
                     "roofline": {k: rf[k] for k in ("bound", "kernel", "achieved", "peak", "unit", "frac")},
                     "plain": ln.get("plain"), "parts": ln.get("parts"), "steps": sub.steps,
                     "seconds": round(time.perf_counter() - t0, 1)}
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


WORKLOADS = {"nested": bench_nested, "dot": bench_dot, "nbody": bench_nbody, "kmeans": bench_kmeans,
             "batched": bench_batched, "expr": bench_expr, "parboil": bench_parboil}


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--gpus", type=int, default=1)
    # 200 warm-up steps (about 0.1 s of the nested step): the GPU's clocks
    # rise during the first milliseconds of work after idle, and a timed
    # region that starts a few steps in measured the nested step ~10 % slower
    # than its steady state
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=200)
    p.add_argument("--workload", choices=sorted(WORKLOADS), default="nested")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-suite", action="store_true",
                   help="default workload only: skip the dot / nbody / kmeans / batched sub-results")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run mx_copy32 over MIB MiB five times (the reference kernel that scales the "
                        "FETCH_SIZE / WRITE_SIZE counters to bytes) and print its size")
    args = p.parse_args(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "multi-GPU runs are not implemented.", file=sys.stderr, flush=True)
        return 2
    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        line = copy_calibration(args.copy_calibration)
    else:
        line = WORKLOADS[args.workload](args)
        if args.workload == "nested" and not args.no_suite:
            torch.cuda.empty_cache()
            line["suite"] = suite_results(args)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
