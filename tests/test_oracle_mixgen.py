"""The oracle's mixture generation (Section 7): DP-means on points,
DP-vMF-means on bearing vectors, and the maximum-likelihood fits.

Pins: passes worked out by hand on a five-point example; separated blobs
recovered exactly; the limits of the threshold (one cluster at the mean,
every point its own cluster); the DP-means objective never rising from one
pass to the next (the property Kulis and Jordan prove); the vMF
concentration against closed-form values of A3(k) = coth k - 1/k; the
isotropic standard deviation against numpy.
"""
import math

import numpy as np
import pytest

import oracle
from synth import points


def test_dpmeans_hand_worked_passes():
    # 1-D points on the x axis, lambda = 1.  Pass 1 starts from the mean 4.06:
    #   0    : d^2 = 16.48 > 1          -> new cluster 1 at 0
    #   0.1  : nearest cluster 1 (0.01)  -> 1
    #   5    : cluster 0 (0.8836)        -> 0
    #   5.2  : cluster 0 (1.2996) > 1    -> new cluster 2 at 5.2
    #   10   : nearest cluster 2 (23.04) -> new cluster 3 at 10
    # centres {5}, {0.05}, {5.2}, {10}; pass 2 changes nothing.
    x = np.zeros((5, 3))
    x[:, 0] = [0.0, 0.1, 5.0, 5.2, 10.0]
    out = oracle.dpmeans(x, 1.0)
    assert out["K"] == 4 and out["passes"] == 2
    assert list(out["labels"]) == [1, 1, 0, 2, 3]
    assert np.allclose(out["centres"][:, 0], [5.0, 0.05, 5.2, 10.0], rtol=0, atol=1e-15)
    assert list(out["counts"]) == [1, 2, 1, 1]
    # one pass only: the centres after the first pass are the same
    one = oracle.dpmeans(x, 1.0, max_passes=1)
    assert one["K"] == 4 and one["passes"] == 1 and list(one["labels"]) == [1, 1, 0, 2, 3]


def test_dpmeans_removes_emptied_clusters():
    # two groups around -5 and 5, lambda = 1; pass 1 starts from the mean 0:
    # -5 opens cluster 1, -5.1 joins it, 5 (d^2 25 from cluster 0, 100 from
    # cluster 1) opens cluster 2, 5.1 joins it.  Cluster 0 is left empty and
    # is removed: clusters 1, 2 become 0, 1 with centres -5.05, 5.05.
    x = np.zeros((4, 3))
    x[:, 0] = [-5.0, -5.1, 5.0, 5.1]
    out = oracle.dpmeans(x, 1.0)
    assert out["K"] == 2 and out["passes"] == 2
    assert list(out["labels"]) == [0, 0, 1, 1]
    assert np.allclose(out["centres"][:, 0], [-5.05, 5.05], rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_dpmeans_recovers_separated_blobs(seed):
    x, lab = points.blobs(7, 150, spread=5.0, radius=0.3, seed=seed)
    out = oracle.dpmeans(x, 1.0)
    assert out["K"] == 7
    # the partition equals the blobs (labels up to renaming)
    pairs = set(zip(out["labels"].tolist(), lab.tolist()))
    assert len(pairs) == 7
    for c in range(7):
        m = out["labels"] == c
        assert np.allclose(out["centres"][c], x[m].mean(axis=0), rtol=0, atol=1e-12)


def test_dpmeans_threshold_limits():
    x, _ = points.blobs(4, 20, spread=3.0, radius=0.5, seed=3)
    d2max = max(np.sum((a - b) ** 2) for a in x for b in x)
    out = oracle.dpmeans(x, d2max * 4)
    assert out["K"] == 1
    assert np.allclose(out["centres"][0], x.mean(axis=0), rtol=0, atol=1e-12)
    d2min = min(np.sum((x[i] - x[j]) ** 2) for i in range(len(x)) for j in range(i))
    out = oracle.dpmeans(x, d2min / 4)
    assert out["K"] == len(x)
    assert sorted(out["counts"].tolist()) == [1] * len(x)


def test_dpmeans_objective_never_rises():
    pc, _ = points.blobs(12, 40, spread=1.2, radius=0.8, seed=5)
    lam = 1.5
    prev = math.inf
    for p in range(1, 12):
        out = oracle.dpmeans(pc, lam, max_passes=p)
        J = np.sum((pc - out["centres"][out["labels"]]) ** 2) + lam * out["K"]
        assert J <= prev + 1e-9
        prev = J
        if out["passes"] < p:
            break


@pytest.mark.parametrize("seed", [0, 1])
def test_dpvmf_recovers_separated_directions(seed):
    d, lab = points.direction_blobs(6, 200, max_angle_deg=4.0, seed=seed)
    out = oracle.dpvmf_means(d, math.cos(math.radians(15)))
    assert out["K"] == 6
    assert len(set(zip(out["labels"].tolist(), lab.tolist()))) == 6
    for c in range(6):
        s = d[out["labels"] == c].sum(axis=0)
        assert np.allclose(out["centres"][c], s / np.linalg.norm(s), rtol=0, atol=1e-12)


def test_dpvmf_threshold_limits():
    d, _ = points.direction_blobs(3, 30, max_angle_deg=10.0, seed=2)
    out = oracle.dpvmf_means(d, -1.5)          # no cosine is below -1.5
    assert out["K"] == 1
    s = d.sum(axis=0)
    assert np.allclose(out["centres"][0], s / np.linalg.norm(s), rtol=0, atol=1e-12)
    out = oracle.dpvmf_means(d, 1.5)           # every cosine is below 1.5: one cluster per direction
    assert out["K"] == len(d)


def test_vmf_kappa_ml_closed_forms():
    def a3(k):
        return 1 / math.tanh(k) - 1 / k
    for k in (1e-3, 0.5, 1.0, 7.0, 50.0, 1e3, 1e5):
        assert oracle.vmf_kappa_ml(a3(k)) == pytest.approx(k, rel=1e-9)
    assert oracle.vmf_kappa_ml(1 / math.tanh(1.0) - 1.0) == pytest.approx(1.0, rel=1e-12)
    # A3(k) = 1 - 1/k exactly in FP64 once coth k rounds to 1
    assert oracle.vmf_kappa_ml(1.0 - 1e-4) == pytest.approx(1e4, rel=1e-10)
    assert oracle.vmf_kappa_ml(0.0) == 0.0 and oracle.vmf_kappa_ml(1.0) == math.inf


def test_gmm_sigma_ml_against_numpy():
    x, lab = points.blobs(5, 60, spread=4.0, radius=0.4, seed=9)
    out = oracle.dpmeans(x, 1.0)
    s = oracle.gmm_sigma_ml(x, out["labels"], out["centres"], out["counts"])
    for c in range(out["K"]):
        m = out["labels"] == c
        assert s[c] == pytest.approx(math.sqrt(np.mean(np.sum((x[m] - x[m].mean(0)) ** 2, axis=1)) / 3), rel=1e-12)


def test_inputs_lie_on_the_grid():
    """The generator's grid makes every FP64 centre sum exact in any order."""
    from synth import scenes
    sc = scenes.cfg2_scene(0)
    pc, _ = points.point_cloud(sc, 20000, seed=1)
    assert np.all(pc / points.POINT_GRID == np.round(pc / points.POINT_GRID))
    assert np.max(np.abs(pc)) < 64.0
    b, _ = points.bearings(sc, pc, 20000, seed=2)
    assert np.all(b / points.DIR_GRID == np.round(b / points.DIR_GRID))
    rng = np.random.default_rng(0)
    perm = rng.permutation(len(pc))
    assert np.array_equal(pc.sum(axis=0), pc[perm].sum(axis=0))
    assert np.sum(pc[:, 0]) == math.fsum(pc[:, 0])
