"""Local minimisation of the oracle's objective (test helper, CPU only).

Several poses can be eps-optimal, so a search result is checked against the
smallest objective value local polishing finds: Nelder-Mead on f(r, t)
(Lemma 1) over the 6-vector (r, t), from the true pose, the pose under test
and seeded random poses of the domain.  Translations outside the domain box
or within zeta of a Gaussian mean (Section 5.1) are rejected.  The objective
is the oracle's, called through ctypes (which releases the GIL, so the
starts run on a thread pool).
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
from scipy.optimize import minimize


def _feasible(sc, t):
    return (np.all(t >= sc.t_lo) and np.all(t <= sc.t_hi) and
            np.min(np.linalg.norm(sc.mu - t, axis=1)) >= sc.zeta)


def random_poses(sc, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        r = rng.uniform(-np.pi, np.pi, 3)
        if np.linalg.norm(r) > np.pi:
            continue
        t = rng.uniform(sc.t_lo, sc.t_hi)
        if _feasible(sc, t):
            out.append(np.concatenate([r, t]))
    return out


def polished_minimum(P, sc, starts, maxfev=(3000,), workers=8):
    """Smallest f found by Nelder-Mead from each start (6-vectors r, t);
    maxfev[k] applies to start k (the last entry to the rest).  Returns
    (f_min, pose, per-start values)."""
    def f(x):
        t = x[3:]
        if not _feasible(sc, t):
            return 1e30
        return P.objective(x[:3], t)[0]

    def run(k):
        x0 = np.asarray(starts[k], dtype=np.float64)
        fev = maxfev[min(k, len(maxfev) - 1)]
        res = minimize(f, x0, method="Nelder-Mead",
                       options={"maxfev": fev, "xatol": 1e-9, "fatol": 1e-13, "adaptive": True,
                                "initial_simplex": x0 + 0.02 * np.vstack([np.zeros(6), np.eye(6)])})
        return min(res.fun, f(x0)), (res.x if res.fun <= f(x0) else x0)

    with ThreadPoolExecutor(workers) as ex:
        out = list(ex.map(run, range(len(starts))))
    vals = [v for v, _ in out]
    k = int(np.argmin(vals))
    return vals[k], out[k][1], vals
