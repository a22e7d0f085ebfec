"""Mixture generation on the GPU (gosma_dpmeans, gosma_dpvmf_means) against
the oracle's serial DP-means / DP-vMF-means and ML fits.

Labels, cluster counts, pass counts and centres are compared bit for bit:
both sides evaluate the same FP64 scores without fused multiply-adds and the
inputs lie on a grid on which the centre sums are exact.  The fitted sigma
(a sum of squares in atomic order) is compared to 1e-12 relative, kappa (a
bisection on coth k - 1/k with the device's tanh) to 1e-12 relative.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1812_01232_amd import Context
from synth import points, scenes

pytestmark = pytest.mark.gpu


def _same(g, o):
    assert g["K"] == o["K"], (g["K"], o["K"])
    assert g["passes"] == o["passes"]
    assert np.array_equal(g["labels"], o["labels"])
    assert np.array_equal(g["counts"], o["counts"])
    assert np.array_equal(g["centres"], o["centres"])


@pytest.mark.parametrize("n,lam,seed,passes", [(1000, 0.5, 1, 100), (20000, 0.8, 2, 100), (100000, 1.0, 3, 20)])
def test_dpmeans_matches_oracle(n, lam, seed, passes):
    sc = scenes.cfg2_scene(0)
    pc, _ = points.point_cloud(sc, n, seed=seed)
    o = oracle.dpmeans(pc, lam, max_passes=passes)
    with Context(0) as ctx:
        g = ctx.dpmeans(pc, lam, max_passes=passes, sigma_min=1e-3)
    _same(g, o)
    s = np.maximum(oracle.gmm_sigma_ml(pc, o["labels"], o["centres"], o["counts"]), 1e-3)
    assert np.allclose(g["spread"], s, rtol=1e-12, atol=0)
    print(f"DP-means n={n}: K={g['K']} in {g['passes']} passes")


@pytest.mark.parametrize("n,deg,seed,passes", [(1000, 8.0, 1, 100), (50000, 10.0, 2, 20), (100000, 8.0, 3, 10)])
def test_dpvmf_matches_oracle(n, deg, seed, passes):
    sc = scenes.cfg2_scene(0)
    pc, _ = points.point_cloud(sc, 50000, seed=seed)
    b, _ = points.bearings(sc, pc, n, seed=seed + 10)
    lam = math.cos(math.radians(deg))
    o = oracle.dpvmf_means(b, lam, max_passes=passes)
    with Context(0) as ctx:
        g = ctx.dpvmf_means(b, lam, max_passes=passes, kappa_max=1e5)
    _same(g, o)
    rbar = np.array([np.linalg.norm(b[o["labels"] == c].sum(axis=0)) / o["counts"][c] for c in range(o["K"])])
    kap = np.array([min(oracle.vmf_kappa_ml(r), 1e5) for r in rbar])
    # kappa solves coth k - 1/k = rbar, whose slope is about 1/k^2 for large k,
    # so an ulp of rbar or of coth moves kappa by about k * 2.2e-16 relative;
    # the bisection stops at a relative width of 1e-15
    tol = (1e-14 + 4e-15 * kap) * kap
    worst = np.max(np.abs(g["spread"] - kap) / tol)
    assert worst <= 1.0, (worst, kap[np.argmax(np.abs(g["spread"] - kap) / tol)])
    print(f"DP-vMF-means n={n}: K={g['K']} in {g['passes']} passes")


def test_cluster_limits_and_errors():
    x, lab = points.blobs(5, 40, spread=4.0, radius=0.3, seed=4)
    with Context(0) as ctx:
        # max_clusters reached: the pass count comes back negated, as in the oracle
        o = oracle.dpmeans(x, 1e-6, max_clusters=8)
        g = ctx.dpmeans(x, 1e-6, max_clusters=8)
        _same(g, o)
        assert g["passes"] < 0
        # one cluster when lambda exceeds every squared distance
        g = ctx.dpmeans(x, 1e9)
        assert g["K"] == 1 and np.array_equal(g["centres"][0], oracle.dpmeans(x, 1e9)["centres"][0])
        from paper_1812_01232_amd.gosma import GosmaError
        with pytest.raises(GosmaError):
            ctx.dpmeans(x, 1.0, max_clusters=0)
        with pytest.raises(GosmaError):
            ctx.dpmeans(x, math.nan)


def test_mixtures_from_data_recover_the_pose():
    """Points and bearings -> mixtures (both clusterings on the GPU) -> the
    search certifies a pose within the success criterion of Section 7."""
    sc = scenes.cfg2_scene(0)
    pc, _ = points.point_cloud(sc, 100000, seed=11)
    b, _ = points.bearings(sc, pc, 100000, seed=12, noise_deg=0.5, outlier_frac=0.2)
    from paper_1812_01232_amd.mixtures import mixtures_from_data
    with Context(0) as ctx:
        mix = mixtures_from_data(ctx, pc, b, lam_points=1.5, cos_lam_bearings=math.cos(math.radians(15.0)),
                                 max_passes=30)
        gen = scenes.Scene(**{**sc.__dict__, **mix, "label1": None, "label2": None, "inlier_src": None})
        ctx.set_scene(gen)
        r = ctx.solve(1e-2, batch_parents=4096, max_queue=1 << 27, time_limit_s=60, sma_iters=100,
                      allow_overflow=True)
    R = oracle.rodrigues(np.asarray(r["r"]))
    ang = math.acos(np.clip((np.trace(R.T @ sc.R_gt) - 1) / 2, -1, 1))
    terr = np.linalg.norm(np.asarray(r["t"]) - sc.t_gt)
    print(f"generated {gen.M}x{gen.N} mixtures; status {r['status']} in {r['seconds']:.2f} s; "
          f"rotation error {math.degrees(ang):.2f} deg, translation error {terr:.3f} m")
    assert ang < 0.1
    assert terr < 0.05 * np.linalg.norm(np.mean(sc.mu, axis=0) - sc.t_gt) + 0.1
