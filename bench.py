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

Also reported: the roofline of the dominant kernel (GMM-vMF pair sums and
bounds) from its HIP-event launch times in the search and the operation
counts of the bound formulas; the bound kernels alone on a 32,768-cube batch;
the FP64 CPU oracle's bound rate on a sample of the same batch with all host
cores and with one; time to eps on the 16 x 16 scene; and time to eps on
fresh 64 x 64 scenes with plain and learned queue order (network trained on
records logged by the search itself).
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

# Operation counts of the bound formulas (profiles/opcount.md, checked by
# tests/test_opcount.py): (plain ops, FMAs among them, transcendentals) per
# work unit.  FLOPs count an FMA as 2; issue slots count a plain op as one
# slot per lane and a transcendental as TRANS_SLOTS (measured 1.8-1.9 on
# gfx950, so 2; a weight of 4, the quarter-rate figure, is reported beside).
OPS = {
    "PAIR12": (100, 15, 15),     # GMM-vMF pair evaluated: UB term (eq. 12) + upper term over the cube (eq. 25, R3)
    "SCREEN12": (8, 4, 0),       # GMM-vMF pair screened
    "PAIR11": (69, 13, 10),      # GMM-GMM pair evaluated: UB term (eq. 11) + lower term (eq. 24, R3)
    "SCREEN11": (7, 3, 0),       # GMM-GMM pair screened
    "CUBE": (116, 30, 3),        # per live cube: decode, Rodrigues, Jacobian corners, ball test
    "ROT_PREP": (72, 22, 5),     # per component and live cube: rotated direction, Lemma 2, screen row
    "TRANS_PREP": (234, 42, 15), # per component and translation cell: kappa interval, Lemma 3, normalisers
}
TRANS_SLOTS = 2
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9            # CUs x SIMDs x lanes x clock
PEAK_FP32_TFLOPS = 157.3


def op_totals(units, trans_slots=TRANS_SLOTS):
    """(FLOPs, issue slots) of {OPS name: count}."""
    flops = slots = 0.0
    for name, n in units.items():
        plain, fma, trans = OPS[name]
        flops += n * (plain + fma + trans)
        slots += n * (plain + trans_slots * trans)
    return flops, slots


def s12_units(w, M):
    """Algorithmic work of the GMM-vMF kernel for work counts w (one problem of M components)."""
    return {"CUBE": w["cubes"], "ROT_PREP": w["cubes"] * M, "SCREEN12": w["s12_screened"],
            "PAIR12": w["s12_evaluated"]}


def s11_units(w, M):
    """Algorithmic work of the GMM-GMM kernel: the translation preparation and the
    pairs, once per distinct translation cell."""
    return {"TRANS_PREP": w["cells"] * M, "SCREEN11": w["s11_screened"], "PAIR11": w["s11_evaluated"]}


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
    """Host cores available to this process: its CPU affinity, capped at the
    OpenMP thread count the environment sets (the host's CPU share for the GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    return min(n, int(omp)) if omp.isdigit() and int(omp) > 0 else n


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
    # and the work counts of the bound kernels
    ctx.get_timing()
    ctx.get_work_counts()
    ctx.set_timing(True)
    ctx.solve(1e-9, max_iters=total, **kw)
    ctx.set_timing(False)
    kt = ctx.get_timing()
    work = ctx.get_work_counts()
    return cubes / dt, dt / steps * 1e3, kt, b, b["max_queue_used"], work


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
    tuned = ctx.autotune(32768, seed=4)
    tiles = {"all": tuned["chosen"], "size_buckets": {str(k): v for k, v in tuned["buckets"].items()}}
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
    ctx.get_work_counts()
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
    work = ctx.get_work_counts()
    live = int(((fl.cpu().numpy() & 6) == 0).sum())
    return BATCH * reps / (e0.elapsed_time(e1) / 1e3), kt, live, work, (rk_np, tk_np)


def cpu_baseline(scene, rk, tk):
    """The FP64 oracle's bound evaluation (Theorem 1) on leading cubes of the
    same 32,768-cube batch the bound-only GPU rate uses: with all host cores,
    then with one.  Samples are sized for about 10-20 s of CPU work."""
    import oracle
    P = oracle.OracleProblem(scene)
    out = {}
    for label, cores in (("all", host_cores()), ("one", 1)):
        # calibrate on a small slice, then time a slice of about 6 s
        t0 = time.perf_counter()
        P.bounds(rk[:64], tk[:64], nthreads=cores)
        per = (time.perf_counter() - t0) / 64
        n = int(min(len(rk), max(256, 6.0 / max(per, 1e-9))))
        t0 = time.perf_counter()
        P.bounds(rk[:n], tk[:n], nthreads=cores)
        dt = time.perf_counter() - t0
        out[label] = {"cores": cores, "cubes": n, "seconds": dt, "value": n / dt}
    a = out["all"]
    return {"value": a["value"], "unit": "cube-bounds/s", "cores": a["cores"], "kind": "oracle",
            "sample": f"oracle bounds (FP64, OpenMP over cubes) of the first {a['cubes']} cubes of the 32,768-cube "
                      f"64x64 batch (rotation levels 2-12, translation levels 1-10) in {a['seconds']:.1f} s on "
                      f"{a['cores']} cores; one core: {out['one']['value']:.0f} cube-bounds/s over "
                      f"{out['one']['cubes']} cubes",
            "one_core": out["one"]}


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
        print(f"records logged: {int(cnt.item())}", file=sys.stderr, flush=True)
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
    # plain_16384: the same search with four times the parents per iteration;
    # plain_sma: with Algorithm 1's SMA step (at most 100 L-BFGS iterations per run)
    variants = (("plain", {}), ("learned", {"order": 1, "learned_window": eps}),
                ("learned_unclamped", {"order": 1}), ("plain_16384", {"batch_parents": 4 * BATCH_PARENTS}),
                ("plain_sma", {"sma_iters": 100}))
    for k in range(n_eval):
        sc = scenes.cfg2_scene(seed=5000 + k)
        ctx.set_scene(sc)
        row = {"seed": 5000 + k}
        for name, kw in variants:
            kw = {"batch_parents": BATCH_PARENTS, **kw}
            r = ctx.solve(eps, max_queue=1 << 29, time_limit_s=time_cap, allow_overflow=True, **kw)
            row[name] = {"status": r["status"], "seconds": r["seconds"], "cubes": r["cubes"],
                         "f_norm": r["f_norm_best"], "lb_norm": r["lb_norm"], "iters": r["iters"]}
            print(f"scene {5000 + k} {name}: status {r['status']} {r['seconds']:.2f} s {r['cubes']} cubes",
                  file=sys.stderr, flush=True)
            if kw.get("sma_iters"):
                row[name].update(sma_runs=r["sma_runs"], sma_improved=r["sma_improved"])
        out["scenes"].append(row)
    # status 0 = eps-certified; 2 = time cap; 3 = queue capacity (both uncertified)
    q = lambda a: [float(x) for x in np.percentile(a, [25, 50, 75])] if len(a) else None
    for name, _ in variants:
        t = np.array([s[name]["seconds"] for s in out["scenes"] if s[name]["status"] == 0])
        out[f"{name}_certified"] = int(t.size)
        out[f"{name}_median_s_certified"] = float(np.median(t)) if t.size else None
        if name != "plain":
            # per scene where both certify: this variant over plain (quartiles)
            both = [s for s in out["scenes"] if s[name]["status"] == 0 and s["plain"]["status"] == 0]
            out[f"{name}_over_plain_time_q1_med_q3"] = q([s[name]["seconds"] / s["plain"]["seconds"] for s in both])
            out[f"{name}_over_plain_cubes_q1_med_q3"] = q([s[name]["cubes"] / s["plain"]["cubes"] for s in both])
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
    ap.add_argument("--kappa-pieces", action="store_true",
                    help="also time the searches with the kappa interval of the S12 upper term in 1, 2 and 4 pieces")
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
    value, ms_step, kt_search, r_search, queue, work_search = search_rate(ctx, args.steps, args.warmup)
    torch.cuda.synchronize()

    # roofline of the GMM-vMF pair kernel over its launches in the search
    # (HIP events on its stream), with the algorithmic work of the formulas
    # (profiles/opcount.md) times the work counts of the same launches
    s12_ms, s12_n = kt_search["s12"]
    s11_ms, s11_n = kt_search["s11"]
    w = work_search
    fl12, sl12 = op_totals(s12_units(w, M))
    _, sl12_4 = op_totals(s12_units(w, M), trans_slots=4)
    fl11, sl11 = op_totals(s11_units(w, M))
    achieved = sl12 / (s12_ms / 1e3) / 1e12
    peak = PEAK_SLOTS / 1e12
    steps_timed = args.warmup + args.steps
    # pair terms: two per evaluated pair (upper and lower bound), S11 once per
    # distinct translation cell with its M diagonal terms; screened-out pairs
    # are not counted
    terms_per_step = 2 * (w["s12_evaluated"] + w["s11_evaluated"] + w["cells"] * M) / steps_timed

    # bound kernels alone on a fixed batch of cubes across levels
    krate, kt, live, work_k, (rk_np, tk_np) = kernel_rate(ctx, scene, 10)

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
        "pair_terms_per_s": terms_per_step / (ms_step / 1e3),
        "pair_terms_per_step": terms_per_step,
        "search_kernels_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in kt_search.items() if v[1]},
        "work_counts_timed_search": dict(w, iterations=steps_timed),
        "bound_kernels_only": {"cube_bounds_per_s": krate, "live_cubes": live,
                               "pairs_evaluated_frac": work_k["s12_evaluated"] / max(work_k["s12_screened"], 1),
                               "ms_per_launch": {"s12": kt["s12"][0] / kt["s12"][1], "s11": kt["s11"][0] / kt["s11"][1]}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                     "frac": achieved / peak, "traffic": measured_traffic(), "traffic_unit": "bytes/launch",
                     "kernel": "k_s12 (GMM-vMF pair sums and bounds), its launches in the search",
                     "launches": s12_n, "ms_per_launch": s12_ms / s12_n,
                     "op_model": "profiles/opcount.md (formula counts x work counts; transcendental = "
                                 f"{TRANS_SLOTS} slots)",
                     "frac_trans_weight_4": sl12_4 / (s12_ms / 1e3) / PEAK_SLOTS,
                     "fp32_tflops": fl12 / (s12_ms / 1e3) / 1e12, "fp32_peak_tflops": PEAK_FP32_TFLOPS,
                     "fp32_frac": fl12 / (s12_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS,
                     "s11": {"ms_per_launch": s11_ms / max(s11_n, 1),
                             "frac": sl11 / (s11_ms / 1e3) / PEAK_SLOTS if s11_ms > 0 else None,
                             "fp32_frac": fl11 / (s11_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS if s11_ms > 0 else None}},
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
    if args.kappa_pieces:
        # the tighter reading of the kappa dependence: cubes and time to eps
        # with the S12 upper term's kappa interval in 1, 2 and 4 pieces
        study = {}
        for name, scn, eps, bp in (("16x16", scenes.cfg1_scene(0), 1e-3, 65536),
                                   ("64x64_5003", scenes.cfg2_scene(seed=5003), 1e-2, BATCH_PARENTS),
                                   ("64x64_5000", scenes.cfg2_scene(seed=5000), 1e-2, BATCH_PARENTS)):
            ctx.set_scene(scn)
            study[name] = {}
            for m in (1, 2, 4):
                ctx.set_kappa_pieces(m)
                r = ctx.solve(eps, batch_parents=bp, max_queue=1 << 28, time_limit_s=60)
                study[name][f"pieces_{m}"] = {"eps": eps, "status": r["status"], "seconds": r["seconds"],
                                              "cubes": r["cubes"], "f_norm": r["f_norm_best"],
                                              "lb_norm": r["lb_norm"]}
                print(f"kappa pieces {m} on {name}: {r['seconds']:.2f} s, {r['cubes']} cubes", file=sys.stderr,
                      flush=True)
            ctx.set_kappa_pieces(1)
        rec["kappa_pieces_study"] = study
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(scene, rk_np, tk_np)
    ctx.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
