"""Benchmark: sub-cube bounds per second of the GOSMA branch-and-bound at
64 x 64 components on one MI355X, and time to the eps-optimum with the plain
best-first queue order against the learned order.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-solve]

Workload (64 x 64, the paper-like scene): 64 Gaussians in a 10 x 10 x 3 m
room; 45 projected inliers with 1 degree noise + 19 outlier directions;
translation domain [-1, 1]^3 m, full rotation ball; 4,096 parents popped per
iteration, i.e. 32,768 sub-cubes bounded per step.

A step is one iteration of the search: select the k lowest-bound cubes,
branch, bound every child (translation-cell sums, GMM-vMF sums, both bounds
of Theorem 1), update d*, prune and push.  `value` = cubes bounded per second
over K steps after W warmup steps of the same search, inputs resident in HBM.

Also reported: the bound kernels alone on a 32,768-cube batch, with the
roofline of the dominant kernel (GMM-vMF pair sums) from its HIP-event launch
times and the op model below; the FP64 CPU oracle's own search rate on
the host's cores; time to eps on the 16 x 16 scene; and time to eps on fresh
64 x 64 scenes with plain and learned queue order (network trained on records
logged by the search itself).
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

# Op model of the GMM-vMF pair kernel, counted from its source.  A plain FP32
# or FP64 operation takes one issue slot per lane (the FP64 vector peak,
# 78.6 TFLOP/s, is one FMA per lane per clock, like unpacked FP32); a
# transcendental (sqrt, rcp, exp2, log2) issues at half that rate on gfx950
# (measured 1.8-1.9 plain-op slots), so it counts 2.
#   per component and cube (the set-up of Lemmas 2-3 and of the kappa
#   interval): 54 FP64 + 409 plain FP32 + 17 transcendentals;
#   per same-class pair screened: 7 plain (a dot product, three threshold
#   terms, a compare);
#   per pair evaluated in full: 125 plain + 14 transcendentals.
TRANS_SLOTS, FP64_SLOTS = 2, 1
PREP_SLOTS = 54 * FP64_SLOTS + 409 + 17 * TRANS_SLOTS
PREP_FLOPS = 54 + 409 + 17
SCREEN_SLOTS, SCREEN_FLOPS = 7, 7 + 4      # 4 of the screen's operations are FMAs
S12_PLAIN, S12_TRANS = 125, 14
S12_SLOTS = S12_PLAIN + TRANS_SLOTS * S12_TRANS
S12_FLOPS = S12_PLAIN + S12_TRANS + 13      # 13 of the plain operations are FMAs
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9            # CUs x SIMDs x lanes x clock
PEAK_FP32_TFLOPS = 157.3
BATCH_PARENTS = 4096
BATCH = 8 * BATCH_PARENTS


def kernel_code_hash(path):
    """SHA-256 of a source file's code: comments removed, whitespace collapsed."""
    import hashlib
    import re
    with open(path) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = re.sub(r"\s+", " ", src).strip()
    return hashlib.sha256(src.encode()).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the bound kernel from the committed counter
    summary, or None once the kernel code differs from the one measured."""
    prof = os.path.join(ROOT, "profiles", "k_s12_64x64_pmc.md")
    src = os.path.join(ROOT, "paper_1812_01232_amd", "csrc", "bound.hip")
    try:
        fields = dict(line.strip().split("=", 1) for line in open(prof) if "=" in line and " " not in line.strip())
        if fields.get("bound_hip_code_sha256") == kernel_code_hash(src):
            return int(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        pass
    return None


def copy_calibration(mib):
    """A plain device copy of `mib` MiB, three times (for scaling byte counters)."""
    import torch
    n = (mib << 20) // 4
    a = torch.zeros(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "launches": 3}), flush=True)


def host_cores():
    try:
        return min(16, len(os.sched_getaffinity(0)))
    except AttributeError:
        return min(16, os.cpu_count() or 1)


def search_rate(ctx, steps, warmup):
    """Cubes bounded per second over `steps` iterations of the search after
    `warmup` iterations, on the product path (captured iteration graph, status
    read back every few iterations).  Two searches from the root, of `warmup`
    and `warmup + steps` iterations; the rate is the difference of their
    bounded-cube counts over the difference of their wall times."""
    total = warmup + steps
    kw = dict(batch_parents=BATCH_PARENTS, max_queue=1 << 27)
    ctx.solve(1e-9, max_iters=warmup, **kw)            # captures the iteration graph
    a = ctx.solve(1e-9, max_iters=warmup, **kw)
    b = ctx.solve(1e-9, max_iters=total, **kw)
    assert a["iters"] == warmup and b["iters"] == total, (a["iters"], b["iters"])
    dt = b["seconds"] - a["seconds"]
    cubes = b["cubes"] - a["cubes"]
    # per-kernel split of the same iterations (direct launches with HIP events)
    # and the pair counts of the GMM-vMF sums
    ctx.get_timing()
    ctx.get_pair_counts()
    ctx.set_timing(True)
    ctx.solve(1e-9, max_iters=total, **kw)
    ctx.set_timing(False)
    kt = ctx.get_timing()
    pairs = ctx.get_pair_counts()
    return cubes / dt, dt / steps * 1e3, kt, b, b["max_queue_used"], pairs


def other_workload_rates(ctx, warmup=20, steps=40):
    """Search rate on the two other workload shapes, each after the autotuner:
    the 256x256 labelled scene (16,384 parents = 131,072 cubes per step) and
    128 problems with M, N uniform on [16, 256] (2,048 parents each, up to
    2.1 M cubes per step), by the same two-search difference as the main rate."""
    from synth import scenes
    out = {}
    ctx.set_scene(scenes.cfg3_scene(0))
    tiles = ctx.autotune(32768, seed=3)["chosen"]
    kw = dict(batch_parents=16384, max_queue=1 << 27)
    ctx.solve(1e-9, max_iters=warmup, **kw)
    a = ctx.solve(1e-9, max_iters=warmup, **kw)
    b = ctx.solve(1e-9, max_iters=warmup + steps, **kw)
    dt = b["seconds"] - a["seconds"]
    out["labelled_256x256"] = {"cube_bounds_per_s": (b["cubes"] - a["cubes"]) / dt, "ms_per_step": dt / steps * 1e3,
                               "cubes_per_step": (b["cubes"] - a["cubes"]) / steps, "tiles": tiles}
    scs = scenes.batch_scenes(128, seed=4000)
    ctx.set_scenes(scs)
    tiles = ctx.autotune(32768, seed=4)["chosen"]
    kw = dict(batch_parents=2048, max_queue=1 << 21, allow_overflow=True)
    ctx.solve_batch(128, 1e-9, max_iters=warmup, **kw)
    ra = ctx.solve_batch(128, 1e-9, max_iters=warmup, **kw)
    rb = ctx.solve_batch(128, 1e-9, max_iters=warmup + steps, **kw)
    dt = rb[0]["seconds"] - ra[0]["seconds"]
    cubes = sum(r["cubes"] for r in rb) - sum(r["cubes"] for r in ra)
    pairs = sum((r1["cubes"] - r0["cubes"]) * (s.M * s.N + s.M * (s.M - 1) // 2) for r0, r1, s in zip(ra, rb, scs))
    out["batch_128"] = {"cube_bounds_per_s": cubes / dt, "ms_per_step": dt / steps * 1e3, "cubes_per_step": cubes / steps,
                        "pair_terms_per_s": 2 * pairs / dt, "tiles": tiles}
    return out


def kernel_rate(ctx, scene, reps):
    """Bound kernels alone on one 32,768-cube batch (cells across levels 2-12 / 1-10)."""
    import torch
    from synth import scenes
    dev = torch.device("cuda", 0)
    rk_np, tk_np = scenes.random_cubes(scene, BATCH, 2600, r_levels=(2, 12), t_levels=(1, 10))
    rk = torch.from_numpy(rk_np.view(np.int64)).to(dev)
    tk = torch.from_numpy(tk_np.view(np.int64)).to(dev)
    ub = torch.empty(BATCH, dtype=torch.float64, device=dev)
    lb = torch.empty(BATCH, dtype=torch.float64, device=dev)
    fl = torch.empty(BATCH, dtype=torch.uint8, device=dev)
    for _ in range(2):
        ctx.eval_bounds(rk, tk, ub, lb, fl)
    torch.cuda.synchronize()
    ctx.get_timing()
    ctx.get_pair_counts()
    ctx.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.eval_bounds(rk, tk, ub, lb, fl)
    e1.record()
    torch.cuda.synchronize()
    ctx.set_timing(False)
    kt = ctx.get_timing()
    pairs = ctx.get_pair_counts()
    live = int(((fl.cpu().numpy() & 6) == 0).sum())
    return BATCH * reps / (e0.elapsed_time(e1) / 1e3), kt, live, pairs


def cpu_baseline(scene, budget_s=15.0):
    """The FP64 oracle's own branch-and-bound on the same scene, bounded in time."""
    import oracle
    P = oracle.OracleProblem(scene)
    cores = host_cores()
    r = P.solve(1e-9, BATCH_PARENTS, time_limit_s=budget_s, nthreads=cores)
    return {"value": r["cubes"] / r["seconds"], "unit": "cube-bounds/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle best-first search on the same 64x64 scene and batch size, stopped after "
                      f"{r['seconds']:.1f} s ({r['cubes']} cubes, {r['iters']} iterations)"}


def learned_comparison(ctx, n_eval, eps, records_cap, epochs, time_cap):
    """Log records from searches, train the network on them, then time to eps
    with plain and learned order on fresh 64x64 scenes."""
    import torch
    from paper_1812_01232_amd.gosma import GosmaError
    from synth import scenes
    QUEUE_OVERFLOW = -4
    dev = torch.device("cuda", 0)
    recs = torch.zeros((records_cap, 21), dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    ctx.set_record_sink(recs, cnt)
    t0 = time.perf_counter()
    i = 0
    while int(cnt.item()) < records_cap and i < 12:
        for sc in (scenes.cfg1_scene(10 + i), scenes.cfg2_scene(10 + i)):
            ctx.set_scene(sc)
            try:
                ctx.solve(eps, batch_parents=BATCH_PARENTS, max_queue=1 << 27, time_limit_s=6, log_records=1)
            except GosmaError as e:     # a full queue ends the search; its records stay valid
                if e.code != QUEUE_OVERFLOW:
                    raise
        i += 1
    ctx.set_record_sink(None, None)
    n = min(int(cnt.item()), records_cap)
    collect_s = time.perf_counter() - t0
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    perm = torch.randperm(n, device=dev, generator=g)
    ntr = int(0.95 * n)
    tr, te = recs[perm[:ntr]].contiguous(), recs[perm[ntr:]].contiguous()
    ctx.mlp_init(0)
    t0 = time.perf_counter()
    hist = ctx.mlp_train(records=tr, epochs=epochs, batch=4096, lr=1e-3, seed=1)
    train_s = time.perf_counter() - t0
    yp = ctx.mlp_predict(te[:, :20].cpu().numpy())
    yt = te[:, 20].cpu().numpy()
    out = {"records": n, "collect_s": collect_s, "train_s": train_s, "train_loss": [float(h) for h in hist],
           "heldout_mae": float(np.mean(np.abs(yp - yt))), "heldout_mae_mean_predictor": float(np.mean(np.abs(yt - yt.mean()))),
           "eps": eps, "scenes": []}
    # plain / learned at the 64 x 64 workload's 4,096 parents per iteration;
    # plain_16384: the same search with four times the parents per iteration
    variants = (("plain", {}), ("learned", {"order": 1, "learned_window": eps}),
                ("learned_unclamped", {"order": 1}), ("plain_16384", {"batch_parents": 4 * BATCH_PARENTS}))
    for k in range(n_eval):
        sc = scenes.cfg2_scene(seed=5000 + k)
        ctx.set_scene(sc)
        row = {"seed": 5000 + k}
        for name, kw in variants:
            kw = {"batch_parents": BATCH_PARENTS, **kw}
            r = ctx.solve(eps, max_queue=1 << 29, time_limit_s=time_cap, allow_overflow=True, **kw)
            row[name] = {"status": r["status"], "seconds": r["seconds"], "cubes": r["cubes"],
                         "f_norm": r["f_norm_best"], "lb_norm": r["lb_norm"]}
        out["scenes"].append(row)
    # status 0 = eps-certified; 2 = time cap; 3 = queue capacity (both uncertified)
    for name, _ in variants:
        t = np.array([s[name]["seconds"] for s in out["scenes"] if s[name]["status"] == 0])
        out[f"{name}_certified"] = int(t.size)
        out[f"{name}_median_s_certified"] = float(np.median(t)) if t.size else None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-eps runs")
    ap.add_argument("--no-other", action="store_true", help="skip the 256x256 and 128-problem rates")
    ap.add_argument("--learned-scenes", type=int, default=4)
    ap.add_argument("--records", type=int, default=1_000_000)
    ap.add_argument("--copy-mib", type=int, default=0, help="only run a plain copy of this size (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the search would shard by splitting "
                                   "each iteration's parents across GPUs, with one all-reduce of d* and the "
                                   "lowest bound per iteration; that path is not built)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1812_01232_amd import Context
    from synth import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_mib > 0:
        copy_calibration(args.copy_mib)
        return
    scene = scenes.cfg2_scene(0)
    ctx = Context(0)
    ctx.set_scene(scene)
    M, N = scene.M, scene.N

    # whole hot path: the search itself
    torch.cuda.synchronize()
    value, ms_step, kt_search, r_search, queue, pairs_search = search_rate(ctx, args.steps, args.warmup)
    torch.cuda.synchronize()

    # roofline of the GMM-vMF pair kernel over its launches in the search
    # (HIP events on its stream), with the algorithmic work from the pair counts
    s12_ms, s12_n = kt_search["s12"]
    s12_s = s12_ms / 1e3
    screened, evaluated = pairs_search
    comps = screened // N        # live cubes x M (one problem, no classes: M N pairs per live cube)
    achieved = (comps * PREP_SLOTS + screened * SCREEN_SLOTS + evaluated * S12_SLOTS) / s12_s / 1e12
    tflops = (comps * PREP_FLOPS + screened * SCREEN_FLOPS + evaluated * S12_FLOPS) / s12_s / 1e12
    peak = PEAK_SLOTS / 1e12

    # bound kernels alone on a fixed batch of cubes across levels
    krate, kt, live, pairs_k = kernel_rate(ctx, scene, 10)

    rec = {
        "metric": "sub-cube bounds/s at 64x64 comps; time-to-eps-optimum plain vs learned order",
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
        "config": {"workload": "64x64 paper-like scene (45 noisy inliers + 19 outliers), branch-and-bound with "
                               "4096 parents = 32768 sub-cubes per step",
                   "M": M, "N": N, "batch_cubes": BATCH, "queue_after_steps": queue},
        "pair_terms_per_s": value * (M * N + M * (M - 1) // 2) * 2,
        "search_kernels_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in kt_search.items() if v[1]},
        "bound_kernels_only": {"cube_bounds_per_s": krate, "live_cubes": live,
                               "pairs_evaluated_frac": pairs_k[1] / max(pairs_k[0], 1),
                               "ms_per_launch": {"s12": kt["s12"][0] / kt["s12"][1], "s11": kt["s11"][0] / kt["s11"][1]}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                     "frac": achieved / peak, "traffic": measured_traffic(), "traffic_unit": "bytes/launch",
                     "kernel": "k_s12 (GMM-vMF pair sums), its launches in the search",
                     "launches": s12_n, "ms_per_launch": s12_ms / s12_n,
                     "pairs_screened": screened, "pairs_evaluated": evaluated,
                     "fp32_tflops": tflops, "fp32_peak_tflops": PEAK_FP32_TFLOPS},
    }
    if not args.no_other:
        rec["other_workloads"] = other_workload_rates(ctx)
    if not args.no_solve:
        # the 16 x 16 search to eps = 1e-3, with 65,536 parents per iteration (the
        # fastest of 1,024 ... 65,536 measured; the bounded-cube count hardly
        # depends on it) and with the 64 x 64 workload's 4,096
        sc1 = scenes.cfg1_scene(0)
        ctx.set_scene(sc1)
        rec["time_to_eps_16x16"] = {}
        for bp in (65536, BATCH_PARENTS):
            r1 = ctx.solve(1e-3, batch_parents=bp, max_queue=1 << 28, time_limit_s=120)
            rec["time_to_eps_16x16"][f"parents_{bp}"] = {
                "eps": 1e-3, "status": r1["status"], "seconds": r1["seconds"], "cubes": r1["cubes"],
                "f_norm": r1["f_norm_best"], "lb_norm": r1["lb_norm"]}
        if args.learned_scenes > 0:
            rec["time_to_eps_64x64_plain_vs_learned"] = learned_comparison(
                ctx, args.learned_scenes, 1e-2, args.records, 4, 8.0)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(scene)
    ctx.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
