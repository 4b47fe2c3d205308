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

Other workloads (--workload): dot (fused map2+reduce vs plain), nbody, kmeans,
batched.  Prints one JSON line on stdout; progress goes to stderr.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class PartTimer:
    """HIP events recorded on the launch stream around each part of a step."""

    def __init__(self, names, steps):
        import torch
        self.names = names
        self.ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
                   for _ in range(steps)]
        self.step = 0
        self.i = 0

    def mark(self):
        if self.step < len(self.ev):
            self.ev[self.step][self.i].record()
            self.i += 1

    def next_step(self):
        self.step += 1
        self.i = 0

    def averages_ms(self):
        out = {}
        for k, n in enumerate(self.names):
            ts = [e[k].elapsed_time(e[k + 1]) for e in self.ev]
            out[n] = sum(ts) / len(ts)
        return out


def timed(step, steps, warmup, names):
    """Run warmup steps, then time `steps` steps; returns (ms_per_step, part ms)."""
    import torch
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    pt = PartTimer(names, steps)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        step(pt)
        pt.next_step()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps, pt.averages_ms()


def gbs(nbytes, ms):
    return nbytes / (ms * 1e-3) / 1e9


def cpu_threads():
    return 1  # the oracle is single-threaded


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
    names = ["offsets", "row_sums", "mmr_fwd", "row_sums_adjoint", "mmr_adjoint_A", "mmr_adjoint_B"]

    def make_step(plain):
        seg = abi.mx_segmented_reduce_plain if plain else abi.mx_segmented_reduce
        mmr = abi.mx_map_map_reduce_plain_f32 if plain else abi.mx_map_map_reduce_f32

        def step(pt):
            m = pt.mark if pt else (lambda: None)
            m(); abi.mx_lengths_to_offsets(d["tL"], offsets, ws)
            m(); seg(abi.MX_ADD, d["tv"], offsets, 0.0, rows)
            m(); mmr(0, 0, d["tA"], d["tB"], C)
            m(); abi.mx_segmented_sum_adjoint_f32(d["tg"], offsets, gvals)
            m(); mmr(0, 1, d["tG"], d["tB"], gA)
            m(); mmr(1, 0, d["tA"], d["tG"], gB)
            m()
        return step

    log("nested: fused steps")
    ms, parts = timed(make_step(False), args.steps, args.warmup, names)
    log(f"nested: fused {ms:.3f} ms/step")
    psteps = max(1, min(args.steps, 3))
    pms, pparts = timed(make_step(True), psteps, 1, names)
    log(f"nested: plain {pms:.3f} ms/step")

    elems = 2 * nval + 3 * M * N * K
    flops = 2.0 * M * N * K
    bytes_ = {
        "offsets": 8 * nseg + 8 * (nseg + 1),
        "row_sums": 4 * nval + 8 * (nseg + 1) + 4 * nseg,
        "row_sums_adjoint": 4 * nval + 8 * (nseg + 1) + 4 * nseg,
    }
    detail = {}
    for n in names:
        e = {"us": round(parts[n] * 1e3, 2), "plain_us": round(pparts[n] * 1e3, 2)}
        if n in bytes_:
            e["GB/s"] = round(gbs(bytes_[n], parts[n]), 1)
            e["frac_hbm"] = round(gbs(bytes_[n], parts[n]) / HBM_PEAK_GBS, 4)
        else:
            tf = flops / (parts[n] * 1e-3) / 1e12
            e["TFLOP/s"] = round(tf, 2)
            e["frac_mfma"] = round(tf / FP32_MFMA_PEAK_TFLOPS, 4)
        detail[n] = e
    dom = "mmr_fwd"
    ach = flops / (parts[dom] * 1e-3) / 1e12
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
        "roofline": {"bound": "mfma", "kernel": "k_gemm_mfma<0,0> (dense map-map-reduce forward)",
                     "achieved": round(ach, 2), "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / FP32_MFMA_PEAK_TFLOPS, 4), "traffic": args.traffic},
        "parts": detail,
        "plain": {"ms_per_step": pms, "value": elems / (pms * 1e-3),
                  "fused_speedup": round(pms / ms, 2)},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_nested(d, rows, C, gA, gB, gvals, offsets)
    return line


def cpu_baseline_nested(d, rows, C, gA, gB, gvals, offsets):
    """The oracle on a bounded sample of the same workload, timed on the host."""
    import torch
    import oracle as O
    torch.cuda.synchronize()
    log("nested: cpu baseline (oracle)")
    L, v, A, B, G, g = d["L"], d["v"], d["A"], d["B"], d["G"], d["g_rows"]
    sample_rows = 24
    t0 = time.perf_counter()
    off = O.offsets_from_lengths(L)
    R = O.segmented_reduce(O.ADD, 0.0, v, off)
    gv = O.segmented_sum_adjoint(g, off)
    Cs = O.matmul(A[:sample_rows], B)
    gAs = O.matmul(G[:sample_rows], B, tb=True)
    gBs = O.matmul(A[:, :sample_rows].copy(), G, ta=True)
    secs = time.perf_counter() - t0
    n = len(L) + 2 * int(L.sum()) + 3 * sample_rows * d["B"].shape[1] * A.shape[1]
    # sample parity: the GPU results of the timed run against the oracle's
    ok = bool(np.array_equal(offsets.cpu().numpy(), off))
    S = O.segmented_reduce(O.ADD, 0.0, np.abs(v), off)
    rg = rows.cpu().numpy().astype(np.float64)
    ok &= bool(np.all(np.abs(rg - R) <= 1e-4 * np.maximum(np.abs(R), S / np.sqrt(np.maximum(L, 1)))))
    ok &= bool(np.array_equal(gvals.cpu().numpy(), gv.astype(np.float32)))
    worst = 0.0
    for got, ref, absref in ((C.cpu().numpy()[:sample_rows], Cs, None),
                             (gA.cpu().numpy()[:sample_rows], gAs, None),
                             (gB.cpu().numpy()[:sample_rows], gBs, None)):
        err = np.abs(got - ref) / np.maximum(np.abs(ref), math.sqrt(A.shape[1]) / 4)
        worst = max(worst, float(err.max()))
    ok &= worst <= 1e-4
    return {"value": n / secs, "unit": "elem/s", "cores": cpu_threads(), "kind": "oracle",
            "seconds": round(secs, 2),
            "sample": f"all 65536 row sums and their adjoint, plus {sample_rows} rows of C, dA and dB "
                      f"(2048-long folds) of the 2048^3 products",
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
    names = ["fused_f32", "fused_i32", "plain_map2", "plain_reduce"]

    def step(pt):
        m = pt.mark if pt else (lambda: None)
        m(); abi.mx_map2_reduce(abi.MX_B_MUL, abi.MX_ADD, ta, tb, 0.0, out, ws)
        m(); abi.mx_map2_reduce(abi.MX_B_MUL, abi.MX_ADD, tai, tbi, 0, outi, ws)
        m(); abi.mx_map2(abi.MX_B_MUL, ta, tb, tmp)
        m(); abi.mx_reduce(abi.MX_ADD, tmp, 0.0, out, ws)
        m()

    ms, parts = timed(step, args.steps, args.warmup, names)
    sweep = {}
    for k in (24, 26):
        nn = 1 << k
        x = torch.rand(nn, device=dev)
        y = torch.rand(nn, device=dev)

        def s2(pt, x=x, y=y):
            m = pt.mark if pt else (lambda: None)
            m(); abi.mx_map2_reduce(abi.MX_B_MUL, abi.MX_ADD, x, y, 0.0, out, ws)
            m()
        _, p2 = timed(s2, 20, 3, ["fused"])
        sweep[f"2^{k}"] = {"us": round(p2["fused"] * 1e3, 2), "GB/s": round(gbs(8 * nn, p2["fused"]), 1),
                           "frac_hbm": round(gbs(8 * nn, p2["fused"]) / HBM_PEAK_GBS, 4)}
    fused = parts["fused_f32"]
    plain = parts["plain_map2"] + parts["plain_reduce"]
    return {
        "metric": METRIC, "value": n / (fused * 1e-3), "unit": "elem/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "dot: map2(*)+reduce(+) over two float32 vectors of 2^20 (+ int32 variant)",
                   "n": n},
        "roofline": {"bound": "hbm", "kernel": "k_reduce<F32,ADD,MUL>", "achieved": round(gbs(8 * n, fused), 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs(8 * n, fused) / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "parts": {k: {"us": round(v * 1e3, 2)} for k, v in parts.items()},
        "plain": {"us": round(plain * 1e3, 2), "fused_speedup": round(plain / fused, 2)},
        "sweep": sweep,
    }


WORKLOADS = {"nested": bench_nested, "dot": bench_dot}


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", choices=sorted(WORKLOADS), default="nested")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--traffic", type=float, default=None,
                   help="HBM bytes per launch of the dominant kernel from hardware counters, if known")
    args = p.parse_args(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "multi-GPU runs are not part of this build.", file=sys.stderr, flush=True)
        return 2
    import torch
    torch.cuda.set_device(0)
    line = WORKLOADS[args.workload](args)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
