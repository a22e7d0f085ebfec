"""Benchmark: GOSMA sub-cube bounds per second at 64 x 64 components on one GPU.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--solve]

A step is one pass of the hot path over one 32,768-cube batch of the
64 x 64 workload (the paper-like scene: 45 projected inliers with 1 degree
noise + 19 outliers, translation domain [-1, 1]^3 m, full rotation ball):
for every cube the translation-cell pair sums (S11), the GMM-vMF pair sums
(S12) and both bounds of Theorem 1.  Inputs are resident in HBM before the
timed region.  `value` is cube-bounds/s.  With --solve the line also carries
the time to the eps-optimum of the branch-and-bound, plain best-first
against the learned queue order.

The line carries the roofline of the dominant kernel (GMM-vMF pair sums):
algorithmic VALU issue slots per launch (op model in the design doc) divided by
its average launch time measured with HIP events on its own stream, against
the issue rate of the chip, and the FP64 CPU oracle timed on a bounded sample
of the same batch on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Op model (VALU issue slots; a transcendental = 4 slots, everything else 1).
# Per GMM-vMF pair, upper + lower summand; per unique GMM-GMM pair, both.
S12_PLAIN, S12_TRANS = 90, 8
S11_PLAIN, S11_TRANS = 85, 8
TRANS_SLOTS = 4
S12_SLOTS = S12_PLAIN + TRANS_SLOTS * S12_TRANS
S11_SLOTS = S11_PLAIN + TRANS_SLOTS * S11_TRANS
S12_FLOPS = S12_PLAIN + S12_TRANS + 20      # FMAs counted twice (20 per pair)
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9            # CUs x SIMDs x lanes x clock
PEAK_FP32_TFLOPS = 157.3
BATCH = 32768


def bench_batch(scene, n, seed):
    """A batch shaped like the B&B's: cells from a range of octree levels."""
    from synth import scenes
    return scenes.random_cubes(scene, n, seed, r_levels=(2, 12), t_levels=(1, 10))


def cpu_baseline(scene, rk, tk, budget_s=15.0):
    import oracle
    P = oracle.OracleProblem(scene)
    try:
        cores = min(16, len(os.sched_getaffinity(0)))
    except AttributeError:
        cores = min(16, os.cpu_count() or 1)
    probe = 256
    t = time.perf_counter()
    P.bounds(rk[:probe], tk[:probe], nthreads=cores)
    rate = probe / (time.perf_counter() - t)
    n = int(min(len(rk), max(probe, rate * budget_s)))
    t = time.perf_counter()
    P.bounds(rk[:n], tk[:n], nthreads=cores)
    dt = time.perf_counter() - t
    return {"value": n / dt, "unit": "cube-bounds/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} cubes of the timed 64x64 batch (FP64, OpenMP over cubes, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solve", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU split is design-only "
                                   "(see DESIGN.md)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1812_01232_amd import Context
    from synth import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    scene = scenes.cfg2_scene(0)
    rk_np, tk_np = bench_batch(scene, BATCH, 2600)
    ctx = Context(0)
    ctx.set_scene(scene)
    rk = torch.from_numpy(rk_np.view(np.int64)).to(dev)
    tk = torch.from_numpy(tk_np.view(np.int64)).to(dev)
    ub = torch.empty(BATCH, dtype=torch.float64, device=dev)
    lb = torch.empty(BATCH, dtype=torch.float64, device=dev)
    fl = torch.empty(BATCH, dtype=torch.uint8, device=dev)

    def step():
        ctx.eval_bounds(rk, tk, ub, lb, fl)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.get_timing()
    ctx.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ctx.set_timing(False)
    kt = ctx.get_timing()
    total_ms = e0.elapsed_time(e1)
    ms_step = total_ms / args.steps
    flags = fl.cpu().numpy()
    live = int(((flags & 6) == 0).sum())
    M, N = scene.M, scene.N
    pairs = live * (M * N + M * (M + 1) // 2) * 2
    value = BATCH * args.steps / (total_ms / 1e3)

    s12_ms, s12_n = kt["s12"]
    s11_ms, s11_n = kt["s11"]
    s12_avg_s = s12_ms / s12_n / 1e3
    slots = live * M * N * S12_SLOTS
    achieved = slots / s12_avg_s / 1e12
    peak = PEAK_SLOTS / 1e12
    rec = {
        "metric": "sub-cube bounds/s at 64x64 comps",
        "value": value,
        "unit": "cube-bounds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64x64 paper-like scene (45 noisy inliers + 19 outliers), 32768-cube batch",
                   "M": M, "N": N, "batch_cubes": BATCH, "live_cubes": live},
        "pair_terms_per_s": pairs * args.steps / (total_ms / 1e3),
        "kernels_ms_per_launch": {"s12": s12_ms / s12_n, "s11": s11_ms / s11_n},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "k_s12 (GMM-vMF pair sums)",
                     "fp32_tflops": live * M * N * S12_FLOPS / s12_avg_s / 1e12,
                     "fp32_peak_tflops": PEAK_FP32_TFLOPS},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(scene, rk_np, tk_np)
    ctx.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
