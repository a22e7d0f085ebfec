"""The learned queue order (not part of the paper's method) against plain
best-first on fresh scenes: the network is trained on records the search
itself logs, then both orders solve the same scenes to the same eps.

Asserted: both orders certify the same minimum within eps (pruning and the
stop test use the exact bounds, so the order cannot change the certificate);
the trained network predicts held-out targets better than their mean does.
Reported (printed and returned to the caller of the benchmark): the
learned/plain ratios of time and of cubes bounded to the certificate, and
the iteration at which each order's d* first came within eps of the final
value (from the search trace).
"""
import numpy as np
import pytest
import torch

from paper_1812_01232_amd import Context
from synth import scenes

pytestmark = pytest.mark.gpu

EPS = 1e-2


def _first_within(trace, f_final, eps_f):
    """(iteration, seconds) of the first trace row whose d* is within eps of f_final."""
    for row in trace:
        if row[4] <= f_final + eps_f:
            return int(row[0]), float(row[1])
    return None, None


def test_learned_order_trained_on_logged_records():
    dev = torch.device("cuda", 0)
    cap = 1_000_000
    recs = torch.zeros((cap, 21), dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    with Context(0) as ctx:
        # records logged by searches of the 16 x 16 and 64 x 64 workloads (a full
        # queue ends a search; the records it logged stay valid)
        ctx.set_record_sink(recs, cnt)
        for sc in (scenes.cfg1_scene(10), scenes.cfg2_scene(10), scenes.cfg1_scene(11), scenes.cfg2_scene(11)):
            if int(cnt.item()) >= cap:
                break
            ctx.set_scene(sc)
            ctx.solve(EPS, batch_parents=4096, log_records=1, max_queue=1 << 27, time_limit_s=6, allow_overflow=True)
        ctx.set_record_sink(None, None)
        n = min(int(cnt.item()), cap)
        assert n > 100000
        perm = torch.randperm(n, device=dev, generator=torch.Generator(device=dev).manual_seed(0))
        ntr = int(0.95 * n)
        tr, te = recs[perm[:ntr]].contiguous(), recs[perm[ntr:n]].contiguous()
        ctx.mlp_init(0)
        ctx.mlp_train(records=tr, epochs=4, batch=4096, lr=1e-3, seed=1)
        yp = ctx.mlp_predict(te[:, :20].cpu().numpy())
        yt = te[:, 20].cpu().numpy().astype(np.float64)
        mae, mae0 = float(np.mean(np.abs(yp - yt))), float(np.mean(np.abs(yt - yt.mean())))
        print(f"{n} records; held-out MAE {mae:.4f} (mean predictor {mae0:.4f})", flush=True)
        assert mae < 0.5 * mae0

        rows = []
        for seed in (5003, 5000):
            sc = scenes.cfg2_scene(seed=seed)
            ctx.set_scene(sc)
            S22 = ctx.S22()
            out = {}
            for name, kw in (("plain", {}), ("learned", {"order": 1, "learned_window": EPS})):
                r = ctx.solve(EPS, batch_parents=4096, max_queue=1 << 29, time_limit_s=30, trace_every=1, **kw)
                out[name] = (r, ctx.trace())
            (rp, tp), (rl, tl) = out["plain"], out["learned"]
            assert rp["status"] == 0 and rl["status"] == 0
            assert abs(rp["f_norm_best"] - rl["f_norm_best"]) <= EPS
            assert rl["f_norm_best"] - rl["lb_norm"] <= EPS
            f_final = min(rp["f_best"], rl["f_best"])
            ip, _ = _first_within(tp, f_final, EPS * S22)
            il, _ = _first_within(tl, f_final, EPS * S22)
            rows.append((seed, rl["seconds"] / rp["seconds"], rl["cubes"] / rp["cubes"], ip, il, rp["iters"], rl["iters"]))
        for s, tr_, cr, ip, il, np_, nl in rows:
            print(f"scene {s}: learned/plain time {tr_:.3f}, cubes {cr:.4f}; d* within eps at iteration "
                  f"{ip} (plain, of {np_}) vs {il} (learned, of {nl})", flush=True)
