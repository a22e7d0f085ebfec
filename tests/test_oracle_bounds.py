"""Theorem 1 bounds of the oracle: validity and convergence by brute force.

The lower-bound value is "parity unpinned" (the paper's proof appendix is not
available), so these tests pin what can be pinned: each summand bound against
dense brute-force optimisation over its interval, the whole lower bound
against the minimum of the objective sampled inside the cube, the upper bound
as the objective at the centre, and convergence as cubes shrink.
"""
import math

import numpy as np
import pytest

import oracle
from synth import scenes


def _logZ(x):
    x = np.asarray(x, dtype=np.float64)
    xs = np.maximum(x, 1e-300)
    return np.where(x <= 0, math.log(2.0), xs + np.log(-np.expm1(-2 * xs)) - np.log(xs))


def _g(a, b, th):
    """log Z(K) - log Z(a) - log Z(b), with K - a - b written without cancellation."""
    K = np.sqrt(np.maximum(a * a + b * b + 2 * a * b * np.cos(th), 0))
    x = -4 * a * b * np.sin(0.5 * th) ** 2 / (K + a + b)
    return x + (_logZ(K) - K) - (_logZ(a) - a) - (_logZ(b) - b)


def test_s12_upper_term_bounds_interval_maximum():
    rng = np.random.default_rng(0)
    for _ in range(3000):
        a = math.exp(rng.uniform(0, math.log(3e4)))
        b = math.exp(rng.uniform(0, math.log(3e4)))
        w = 10 ** rng.uniform(-5, 0.5)
        B = rng.uniform(0, math.pi) * rng.uniform() ** 3
        grid = np.linspace(a, a * (1 + w), 401)
        gmax = _g(grid, b, B).max()
        exact = math.exp(gmax)
        bound = oracle.s12_upper_term(a, a * (1 + w), b, B)
        # FP64 rounding of an exponent of size |g|: relative 1e-13 (1 + |g|)
        assert bound >= exact * (1 - 1e-13 * (1 + abs(gmax)))
        if w < 1e-3 and exact > 1e-6:
            assert bound <= exact * (1 + 1e-2)   # tight for small intervals


def test_s12_upper_term_in_pieces():
    """The S12 upper term with the kappa interval split into m pieces (the
    tighter reading of the kappa dependence): one piece is the default term
    bit for bit; the largest of the pieces' expansion bounds lies above the
    ratio's maximum over the interval (dense grid) for every m, and approaches
    it as the pieces shrink (the expansion's error is second order in the
    piece width); the capped term stays above the maximum."""
    rng = np.random.default_rng(11)
    for _ in range(1500):
        a = math.exp(rng.uniform(0, math.log(3e4)))
        b = math.exp(rng.uniform(0, math.log(3e4)))
        w = 10 ** rng.uniform(-4, 0.5)
        B = rng.uniform(0, math.pi) * rng.uniform() ** 3
        ahi = a * (1 + w)
        grid = np.linspace(a, ahi, 2049)
        gmax = _g(grid, b, B).max()
        tol = 1e-13 * (1 + abs(gmax))
        assert oracle.s12_upper_term_pieces(a, ahi, b, B, 1) == oracle.s12_upper_term(a, ahi, b, B)
        gaps = []
        for m in (1, 2, 4, 16, 64):
            e = np.linspace(a, ahi, m + 1)
            e[0], e[-1] = a, ahi
            elog = max(oracle.s12_expansion_log(e[k], e[k + 1], b, B) for k in range(m))
            assert elog >= gmax - tol
            gaps.append(elog - gmax)
            term = oracle.s12_upper_term_pieces(a, ahi, b, B, m)
            assert term >= math.exp(gmax) * (1 - tol)
        # second-order convergence of the expansion (the grid resolves the
        # maximum to (width / 2048)^2 times the curvature bound)
        assert gaps[-1] <= gaps[0] * 0.05 + 1e-9 * (1 + abs(gmax)) + (ahi - a) ** 2 / 3e5


def test_s12_far_apart_bound():
    """For directions far apart the S12 summand bound is at most the smaller of
    2 G(ahi) G(b) exp(-q c) and G(ahi) G(b) exp(-min(q, 2) c) / sqrt(2 alo b)
    (G(y) = y / (1 - e^{-2y}), q = 4 sin^2(B/2), c = alo b / (2 (alo + b))),
    and both expressions bound the ratio Z(K)/(Z(a) Z(b)) over a dense grid
    of concentrations in [alo, ahi] and angles >= B."""
    rng = np.random.default_rng(5)
    G = lambda y: y / -np.expm1(-2 * y)
    active = 0
    for _ in range(2000):
        a = math.exp(rng.uniform(0, math.log(3e4)))
        b = math.exp(rng.uniform(0, math.log(3e4)))
        w = 10 ** rng.uniform(-5, 1.5)
        B = rng.uniform(0, math.pi)
        ahi = a * (1 + w)
        q = 4 * math.sin(0.5 * B) ** 2
        c = a * b / (2 * (a + b))
        l2 = math.log(2 * G(ahi) * G(b)) - q * c
        lK = math.log(G(ahi) * G(b)) - min(q, 2.0) * c - 0.5 * math.log(2 * a * b)
        lfar = min(l2, lK)
        far = math.exp(lfar)
        bound = oracle.s12_upper_term(a, ahi, b, B)
        # FP64 rounding of an exponent of size |log far|, and of log Z(y) - y
        # (the oracle's log G) for y up to ahi
        tol = 1e-13 * (1 + abs(lfar)) + 4e-16 * (ahi + b)
        assert bound <= far * (1 + tol)
        active += bound > 0 and bound >= far * (1 - tol)
        ag = np.linspace(a, ahi, 81)[:, None]
        tg = np.linspace(B, math.pi, 81)[None, :]
        g = _g(ag, b, tg)
        slack = 1e-12 * (1 + np.abs(g).max())
        assert g.max() <= l2 + slack
        assert g.max() <= lK + slack
    assert active > 20


def test_s11_lower_log_bounds_box_minimum():
    rng = np.random.default_rng(1)
    for _ in range(1500):
        a = math.exp(rng.uniform(0, math.log(3e4)))
        b = math.exp(rng.uniform(0, math.log(3e4)))
        wa = 10 ** rng.uniform(-5, 0)
        wb = 10 ** rng.uniform(-5, 0)
        A = rng.uniform(0, math.pi) * rng.uniform() ** 3
        ga = np.linspace(a, a * (1 + wa), 41)[:, None]
        gb = np.linspace(b, b * (1 + wb), 41)[None, :]
        exact = _g(ga, gb, A).min()
        bound = oracle.s11_lower_log(a, a * (1 + wa), b, b * (1 + wb), A)
        assert bound <= exact + 1e-10 * (1 + abs(exact))


def _key_containing(x, lo, hi, L):
    idx = np.floor((np.asarray(x) - lo) / (hi - lo) * (2 ** L)).astype(int)
    idx = np.clip(idx, 0, 2 ** L - 1)
    return int(scenes.pack_key(L, idx[0], idx[1], idx[2]))


def _sampled_min(P, sc, rk, tk, n, rng):
    rc, rh = oracle.decode(rk, sc.r_lo, sc.r_hi)
    tc, th = oracle.decode(tk, sc.t_lo, sc.t_hi)
    best = math.inf
    for q in range(n):
        r = rc + rh * rng.uniform(-1, 1, 3)
        t = tc + th * rng.uniform(-1, 1, 3)
        if q < 64:   # corners and faces too
            r = rc + rh * rng.choice([-1.0, 1.0], 3)
            t = tc + th * rng.choice([-1.0, 1.0], 3)
        if np.min(np.linalg.norm(sc.mu - t, axis=1)) < sc.zeta:
            continue
        best = min(best, P.objective(r, t)[0])
    return best


@pytest.mark.parametrize("seed,M,N,noise", [(31, 5, 5, 0.0), (32, 6, 8, 1.0), (33, 8, 6, 2.0)])
def test_lower_bound_below_sampled_minimum(seed, M, N, noise):
    """lb <= min f over >= 4096 feasible poses sampled in each cube, and
    ub = f(centre), on random small cubes and on cubes around the true pose."""
    sc = scenes.small_scene(M, N, seed=seed, noise_deg=noise, n_inliers=min(M, N) - 1)
    P = oracle.OracleProblem(sc)
    rng = np.random.default_rng(seed)
    rk, tk = scenes.random_cubes(sc, 12, seed + 500, r_levels=(4, 8), t_levels=(2, 6))
    keys = list(zip(rk.tolist(), tk.tolist()))
    for Lr, Lt in [(5, 3), (7, 5), (9, 7), (11, 9)]:
        keys.append((_key_containing(sc.r_gt, sc.r_lo, sc.r_hi, Lr), _key_containing(sc.t_gt, sc.t_lo, sc.t_hi, Lt)))
    b = P.bounds([k[0] for k in keys], [k[1] for k in keys])
    checked = 0
    for q, (rkq, tkq) in enumerate(keys):
        if b["status"][q] != 0:
            continue
        smin = _sampled_min(P, sc, rkq, tkq, 4096, rng)
        if not math.isfinite(smin):
            continue
        assert b["lb"][q] <= smin + 1e-12 * abs(smin)
        rc, _ = oracle.decode(rkq, sc.r_lo, sc.r_hi)
        tc, _ = oracle.decode(tkq, sc.t_lo, sc.t_hi)
        if math.isfinite(b["ub"][q]):
            f, s11, s12 = P.objective(rc, tc)
            assert b["ub"][q] == f
            assert b["s11_ub"][q] == s11 and b["s12_ub"][q] == s12
            assert b["lb"][q] <= b["ub"][q]
        checked += 1
    assert checked >= 8


def test_lower_bound_with_kappa_pieces_stays_valid():
    """With the kappa interval of the S12 upper term in 4 pieces the lower
    bound stays below the objective sampled in each cube, and it is at least
    the one-piece bound on most cubes (its sum can only drop where the
    piecewise expansion replaced a cap)."""
    sc = scenes.small_scene(6, 8, seed=32, noise_deg=1.0, n_inliers=5)
    P = oracle.OracleProblem(sc)
    rng = np.random.default_rng(40)
    rk, tk = scenes.random_cubes(sc, 10, 540, r_levels=(3, 8), t_levels=(1, 6))
    b1 = P.bounds(rk, tk)
    try:
        oracle.set_kappa_pieces(4)
        b4 = P.bounds(rk, tk)
    finally:
        oracle.set_kappa_pieces(1)
    with pytest.raises(ValueError):
        oracle.set_kappa_pieces(0)
    ok = b1["status"] == 0
    assert np.array_equal(b1["ub"][ok], b4["ub"][ok])
    assert np.mean(b4["lb"][ok] >= b1["lb"][ok] - 1e-12 * np.abs(b1["lb"][ok])) >= 0.8
    for q in np.flatnonzero(ok):
        smin = _sampled_min(P, sc, int(rk[q]), int(tk[q]), 4096, rng)
        if math.isfinite(smin):
            assert b4["lb"][q] <= smin + 1e-12 * abs(smin)


def test_bounds_converge_as_cubes_shrink():
    """UB - LB -> 0 as the cube around a pose halves (the B&B requirement
    stated at the start of Section 5)."""
    sc = scenes.small_scene(8, 8, seed=85)
    P = oracle.OracleProblem(sc)
    S22 = P.S22()
    gaps = []
    for Lr, Lt in [(4, 2), (6, 4), (8, 6), (10, 8), (12, 10), (14, 12)]:
        rk = _key_containing(sc.r_gt, sc.r_lo, sc.r_hi, Lr)
        tk = _key_containing(sc.t_gt, sc.t_lo, sc.t_hi, Lt)
        b = P.bounds([rk], [tk])
        gaps.append((b["ub"][0] - b["lb"][0]) / S22)
    assert all(g > 0 for g in gaps)
    assert all(gaps[k + 1] < 0.6 * gaps[k] for k in range(len(gaps) - 1))
    assert gaps[-1] < 2e-3


def test_cube_status_edge_cases():
    sc = scenes.cfg1_scene(0)
    P = oracle.OracleProblem(sc)
    # rotation cell [3pi/4, pi]^3: its nearest point to 0 has norm 3 sqrt(3) pi / 4 > pi
    corner = int(scenes.pack_key(3, 7, 7, 7))
    # translation cell that lies entirely within zeta of a Gaussian mean
    sc2 = scenes.small_scene(4, 4, seed=1)
    sc2.mu[0] = np.array([0.01, 0.02, -0.03])     # inside the translation domain
    P2 = oracle.OracleProblem(sc2)
    inner_t = _key_containing(sc2.mu[0], sc2.t_lo, sc2.t_hi, 6)
    b = P.bounds([corner, 0], [0, 0])
    assert b["status"][0] == 1 and math.isinf(b["lb"][0])
    assert b["status"][1] == 0 and b["lb"][1] < b["ub"][1]
    b2 = P2.bounds([0], [inner_t])
    assert b2["status"][0] == 2 and math.isinf(b2["lb"][0])
    # a cell that touches the ball is kept
    touching = int(scenes.pack_key(1, 1, 1, 1))
    assert P.bounds([touching], [0])["status"][0] == 0


def test_pair_screen_inequality_implies_negligible_summand():
    """The GMM-vMF pair screen of the bound kernel, written out on the CPU: a
    pair is dropped when max(d cos Psi, -sin Psi) <= (1 - sin Psi - Lam/alo)
    - l/b - Lam/b - l/alo with d = cos(theta), Lam = ln(w1 G(ahi)/sqrt(alo)),
    l = ln(w2 G(b)/sqrt(2 b)) - ln(thr).  Whenever it drops a pair, the
    oracle's S12 summand bound at B = max(0, theta - Psi), weighted, and the
    centre summand at any concentration in [alo, ahi] are below thr."""
    rng = np.random.default_rng(7)
    G = lambda y: y / -np.expm1(-2 * y)
    dropped = 0
    for _ in range(4000):
        alo = math.exp(rng.uniform(math.log(2), math.log(2e4)))
        ahi = alo * (1 + 10 ** rng.uniform(-4, 0.5))
        b = math.exp(rng.uniform(math.log(2), math.log(2e4)))
        psi = rng.uniform(0, math.pi / 2) * rng.uniform() ** 2
        theta = rng.uniform(0, math.pi)
        w1, w2 = 10 ** rng.uniform(-3, 0, size=2)
        thr = 10 ** rng.uniform(-14, -6)
        lam = math.log(w1 * G(ahi) / math.sqrt(alo))
        l = math.log(w2 * G(b) / math.sqrt(2 * b)) - math.log(thr)
        d = math.cos(theta)
        rhs = (1 - math.sin(psi) - lam / alo) - l / b - lam / b - l / alo
        if not max(d * math.cos(psi), -math.sin(psi)) <= rhs:
            continue
        dropped += 1
        B = max(0.0, theta - psi)
        assert w1 * w2 * oracle.s12_upper_term(alo, ahi, b, B) <= thr * (1 + 1e-9)
        for a in (alo, 0.5 * (alo + ahi), ahi):
            centre = math.exp(_g(np.array([a]), b, np.array([theta]))[0])
            assert w1 * w2 * centre <= thr * (1 + 1e-9)
    assert dropped > 500


def test_gmm_pair_screen_inequality_implies_negligible_summand():
    """The GMM-GMM pair screen, written out on the CPU: a pair of centre
    concentrations k, k' at angle theta is dropped when
    min(q, 2) k k' >= 2 (Lam + Lam' - ln thr)(k + k'), q = 2 - 2 cos(theta),
    Lam = ln(w G(k)/sqrt(k)) + ln(2)/4.  Whenever it drops a pair, the weighted
    centre summand 2 w w' Z(K)/(Z(k) Z(k')) and the oracle's lower term over
    any box of concentrations around the centre, at any angle >= theta, are
    below thr."""
    rng = np.random.default_rng(8)
    G = lambda y: y / -np.expm1(-2 * y)
    dropped = 0
    for _ in range(4000):
        k1, k2 = np.exp(rng.uniform(math.log(2), math.log(2e4), size=2))
        theta = rng.uniform(0, math.pi)
        w1, w2 = 10 ** rng.uniform(-3, 0, size=2)
        thr = 10 ** rng.uniform(-14, -6)
        lam1 = math.log(w1 * G(k1) / math.sqrt(k1)) + 0.25 * math.log(2)
        lam2 = math.log(w2 * G(k2) / math.sqrt(k2)) + 0.25 * math.log(2)
        q = 2 - 2 * math.cos(theta)
        if not min(q, 2.0) * k1 * k2 >= 2 * (lam1 + lam2 - math.log(thr)) * (k1 + k2):
            continue
        dropped += 1
        centre = math.exp(_g(np.array([k1]), k2, np.array([theta]))[0])
        assert 2 * w1 * w2 * centre <= thr * (1 + 1e-9)
        h1, h2 = k1 * rng.uniform(0, 0.5), k2 * rng.uniform(0, 0.5)
        A = min(math.pi, theta + rng.uniform(0, 0.3))
        lo = oracle.s11_lower_log(k1 - h1, k1 + h1, k2 - h2, k2 + h2, A)
        assert 2 * w1 * w2 * math.exp(lo) <= thr * (1 + 1e-9)
    assert dropped > 500
