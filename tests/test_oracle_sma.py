"""The oracle's objective gradient and SMA local optimiser (Section 6).

Pins, none of which reuses the gradient's own arithmetic:
  * the gradient against central finite differences of the objective (itself
    pinned by sphere quadrature and the zero-distance pose), on unlabelled and
    labelled scenes and on poses near the rotation-angle singularity at 0;
  * SMA never raises f, ends at a point where the finite-difference gradient
    (projected on the box) is small, stays in the box and away from the means,
    and from starts near the true pose of a noise-free scene reaches the closed
    form minimum (zero distance) at the true pose;
  * Algorithm 1 with SMA keeps the eps certificate of the search without it.
"""
import math

import numpy as np
import pytest

import oracle
from synth import scenes


def fd_grad(P, x, h):
    g = np.zeros(6)
    for a in range(6):
        xp, xm = x.copy(), x.copy()
        xp[a] += h
        xm[a] -= h
        g[a] = (P.objective(xp[:3], xp[3:])[0] - P.objective(xm[:3], xm[3:])[0]) / (2 * h)
    return g


@pytest.mark.parametrize("which", ["cfg1", "cfg2", "small_labelled"])
def test_gradient_matches_finite_differences(which):
    if which == "cfg1":
        sc = scenes.cfg1_scene(0)
    elif which == "cfg2":
        sc = scenes.cfg2_scene(0)
    else:
        sc = scenes.small_scene(12, 10, seed=7, noise_deg=1.0, n_inliers=8, n_labels=3)
    P = oracle.OracleProblem(sc)
    rng = np.random.default_rng(11)
    for k in range(6):
        r = sc.r_gt + rng.normal(0, 0.3, 3)
        if k == 0:
            r = rng.normal(0, 1e-5, 3)          # near |r| = 0, where the left Jacobian uses its series
        t = sc.t_gt + rng.normal(0, 0.2, 3)
        f, g = P.objective_grad(r, t)
        assert f == pytest.approx(P.objective(r, t)[0], rel=1e-10, abs=1e-15)   # summation order
        x = np.concatenate([r, t])
        # steps of 1e-4: the objective's own rounding (exponents of size
        # kappa ~ 1e4 cancel) makes smaller steps noisy; the Richardson
        # combination removes the h^2 truncation term
        fd = fd_grad(P, x, 1e-4)
        fd2 = fd_grad(P, x, 2e-4)
        fdr = (4 * fd - fd2) / 3
        scale = np.max(np.abs(fdr)) + 1e-12
        assert np.max(np.abs(g - fdr)) <= 1e-6 * scale, (k, g, fdr)


def test_gradient_single_pair_translation_only():
    """M = N = 1 with the vMF direction along the camera-frame direction: the
    rotation gradient vanishes (the pair is aligned), and the translation
    gradient along the mean's direction is the derivative of the closed-form
    single-pair value, computed here by hand."""
    mu = np.array([[0.0, 0.0, 2.0]])
    sc = scenes.Scene(mu=mu, sigma=np.array([0.2]), phi1=np.array([1.0]), dir2=np.array([[0.0, 0.0, 1.0]]),
                      kappa2=np.array([50.0]), phi2=np.array([1.0]), r_gt=np.zeros(3), R_gt=np.eye(3),
                      t_gt=np.zeros(3), t_lo=np.full(3, -1.0), t_hi=np.full(3, 1.0))
    P = oracle.OracleProblem(sc)
    z = 0.3
    f, g = P.objective_grad(np.zeros(3), np.array([0.0, 0.0, z]))
    assert np.max(np.abs(g[:3])) < 1e-12

    def logZ(x):
        return x + math.log(-math.expm1(-2 * x)) - math.log(x)

    def f_of(z):
        rho = 2.0 - z
        a = rho * rho / 0.04 + 1.0
        b = 50.0
        s11 = math.exp(logZ(2 * a) - 2 * logZ(a))
        s12 = math.exp(logZ(a + b) - logZ(a) - logZ(b))
        return s11 - 2 * s12

    h = 1e-6
    assert g[5] == pytest.approx((f_of(z + h) - f_of(z - h)) / (2 * h), rel=1e-6)
    assert abs(g[3]) < 1e-12 and abs(g[4]) < 1e-12


def test_sma_reaches_true_pose_on_noise_free_scene():
    sc = scenes.cfg1_scene(0)
    P = oracle.OracleProblem(sc)
    S22 = P.S22()
    rng = np.random.default_rng(3)
    for _ in range(3):
        r0 = sc.r_gt + rng.normal(0, 0.05, 3)
        t0 = np.clip(sc.t_gt + rng.normal(0, 0.05, 3), sc.t_lo, sc.t_hi)
        f0 = P.objective(r0, t0)[0]
        out = P.sma(r0, t0, max_iters=200)
        assert out["iters"] > 0
        assert out["f"] <= f0
        # the closed-form minimum: zero distance at the true pose
        assert (out["f"] + S22) / S22 < 1e-6
        assert np.linalg.norm(out["t"] - sc.t_gt) < 1e-3
        R = oracle.rodrigues(out["r"])
        assert math.acos(np.clip((np.trace(R.T @ sc.R_gt) - 1) / 2, -1, 1)) < 1e-3


def test_sma_first_order_optimal_and_monotone():
    sc = scenes.cfg2_scene(0)
    P = oracle.OracleProblem(sc)
    rng = np.random.default_rng(5)
    for _ in range(2):
        r0 = sc.r_gt + rng.normal(0, 0.1, 3)
        t0 = np.clip(sc.t_gt + rng.normal(0, 0.1, 3), sc.t_lo, sc.t_hi)
        f0, s11, s12 = P.objective(r0, t0)
        out = P.sma(r0, t0, max_iters=300, gtol=1e-9, ftol=1e-14)
        assert out["f"] <= f0
        x = np.concatenate([out["r"], out["t"]])
        assert np.all(x[3:] >= sc.t_lo) and np.all(x[3:] <= sc.t_hi)
        assert np.min(np.linalg.norm(sc.mu - x[3:], axis=1)) >= sc.zeta
        g = (4 * fd_grad(P, x, 1e-4) - fd_grad(P, x, 2e-4)) / 3
        g0 = (4 * fd_grad(P, np.concatenate([r0, t0]), 1e-4) - fd_grad(P, np.concatenate([r0, t0]), 2e-4)) / 3
        # f carries rounding of about 1e-12 of S11 (exponents of size kappa
        # cancel), so no step gains once |g|^2 / (2 H) falls to that level,
        # H ~ kappa ~ 1e4: |g| ~ 1e-4 of the scale is the attainable floor
        assert np.max(np.abs(g)) <= 1e-4 * (s11 + 2 * s12)
        assert np.max(np.abs(g)) <= 1e-3 * np.max(np.abs(g0))


def test_sma_respects_the_box():
    """A translation box that excludes the true centre: the result lies on the
    box face nearest to it, and the gradient there points out of the box."""
    sc = scenes.cfg1_scene(0)
    lo = sc.t_lo.copy()
    hi = sc.t_hi.copy()
    hi[0] = sc.t_gt[0] - 0.05          # the true centre lies beyond the +x face
    lo[0] = min(lo[0], hi[0] - 0.5)
    sc2 = scenes.Scene(**{**sc.__dict__, "t_lo": lo, "t_hi": hi})
    P = oracle.OracleProblem(sc2)
    t0 = np.clip(sc.t_gt, lo, hi) - np.array([0.1, 0.0, 0.0])
    out = P.sma(sc.r_gt, t0, max_iters=300, gtol=1e-9, ftol=1e-14)
    assert out["iters"] > 0
    assert out["t"][0] == pytest.approx(hi[0], abs=1e-12)
    _, g = P.objective_grad(out["r"], out["t"])
    assert g[3] < 0          # f still falls towards +x, outside the box


def test_sma_rejects_disallowed_starts():
    sc = scenes.cfg1_scene(0)
    P = oracle.OracleProblem(sc)
    assert P.sma(sc.r_gt, sc.mu[0] + 0.01)["iters"] == -1          # within zeta of a mean
    assert P.sma(sc.r_gt, sc.t_hi + 0.1)["iters"] == -1            # outside the box


@pytest.mark.parametrize("M,N,seed,noise", [(5, 6, 90, 2.0), (4, 4, 81, 0.0)])
def test_solve_with_sma_keeps_the_certificate(M, N, seed, noise):
    sc = scenes.small_scene(M, N, seed=seed, noise_deg=noise, n_inliers=min(M, N) - (1 if noise else 0))
    P = oracle.OracleProblem(sc)
    eps = 1e-2
    a = P.solve(eps, 256, time_limit_s=120)
    b = P.solve(eps, 256, time_limit_s=120, sma_iters=100)
    assert a["status"] == 0 and b["status"] == 0
    assert b["sma_runs"] >= 1
    # both certify the same minimum within eps; SMA's value is a value of f
    assert abs(a["f_norm_best"] - b["f_norm_best"]) <= eps
    assert b["f_norm_best"] - b["lb_norm"] <= eps
    f, _, _ = P.objective(b["r"], b["t"])
    assert f == pytest.approx(b["f_best"], rel=1e-12, abs=1e-15)
    # d* from SMA is at least as good as the best cube centre of the same iteration
    assert b["f_norm_best"] <= a["f_norm_best"] + eps
