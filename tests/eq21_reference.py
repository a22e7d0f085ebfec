"""Plain-numpy evaluation of the lower bound of Theorem 1 (eq. 21) as the paper
states it, by dense sampling.

Test code only.  It shares nothing with the oracle or the HIP library: the
rotation matrices come from scipy's rotation-vector routine, and every
quantity the paper defines as an extremum is taken over dense samples:

  psi_t(mu, C_t)   Lemma 3 / eq. 19: the largest angle between mu - t and
                   mu - t0 over a grid of t covering the cuboid (vertices,
                   edges, faces and interior), or pi when mu lies in C_t;
  psi_r(p, C_r)    Lemma 2 / eq. 18: the largest angle over a grid on the
                   cube's surface, capped at pi.  Eq. 25 pairs it with
                   R_r0^{-1} mu_2j, and the proof's reverse triangle
                   inequality needs the angle between R_r^{-1} mu_2j and
                   R_r0^{-1} mu_2j, so that is the angle sampled;
  min/max over t   each summand of eq. 21 over the feasible translations of
                   C_t (a grid of t, restricted to the domain Omega_t of
                   Section 5.1: at least zeta from every Gaussian mean), with
                   the exact kappa_1i(t) of eq. 13 at each sample.

The diagonal GMM pairs (i = j in the first sum) are taken literally, with
A = min(pi, 2 psi_t) from eq. 24.  Sampling under-estimates every maximum
and over-estimates every minimum, so the value here is, up to the sampling
resolution, at or above the exact value of eq. 21.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial.transform import Rotation


def log_Z(x):
    """log Z(x), Z(x) = (e^x - e^-x)/x (eq. 2), without overflow; Z(0) = 2."""
    x = np.asarray(x, dtype=np.float64)
    xs = np.maximum(x, 1e-300)
    return np.where(x <= 0, math.log(2.0), xs + np.log(-np.expm1(-2.0 * xs)) - np.log(xs))


def log_ratio(a, b, theta):
    """log Z(K) - log Z(a) - log Z(b) with K^2 = a^2 + b^2 + 2 a b cos(theta)
    (eqs. 11-12, 22-23); K - a - b is formed as -4 a b sin^2(theta/2)/(K + a + b)."""
    a, b, theta = np.broadcast_arrays(np.asarray(a, float), np.asarray(b, float), np.asarray(theta, float))
    q = 4.0 * np.sin(0.5 * theta) ** 2
    K = np.sqrt(np.maximum((a + b) ** 2 - a * b * q, 0.0))
    x = -a * b * q / (K + a + b)
    ell = lambda y: log_Z(y) - y
    return x + ell(K) - ell(a) - ell(b)


def angle(u, v):
    """Angle between vectors along the last axis, atan2(|u x v|, u . v)."""
    return np.arctan2(np.linalg.norm(np.cross(u, v), axis=-1), np.sum(u * v, axis=-1))


def class_weights(scene):
    """Weights renormalised within each class and the class factor 1/|Lambda| (eq. 17)."""
    l1 = scene.label1 if scene.label1 is not None else np.zeros(scene.M, int)
    l2 = scene.label2 if scene.label2 is not None else np.zeros(scene.N, int)
    w1 = np.array(scene.phi1, float)
    w2 = np.array(scene.phi2, float)
    for c in np.unique(np.concatenate([l1, l2])):
        s1, s2 = w1[l1 == c].sum(), w2[l2 == c].sum()
        w1[l1 == c] /= s1 if s1 > 0 else 1.0
        w2[l2 == c] /= s2 if s2 > 0 else 1.0
    return w1, w2, l1, l2, 1.0 / max(scene.n_labels, 1)


def box_grid(centre, half, n):
    """n^3 points on a regular grid spanning the box (its corners included)."""
    axes = [np.linspace(c - h, c + h, n) for c, h in zip(centre, half)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
    return g.reshape(-1, 3)


def surface_grid(centre, half, n):
    """n x n points on each of the six faces of the box."""
    s = np.linspace(-1.0, 1.0, n)
    a, b = np.meshgrid(s, s, indexing="ij")
    a, b = a.ravel(), b.ravel()
    pts = []
    for ax in range(3):
        o1, o2 = [k for k in range(3) if k != ax]
        for side in (-1.0, 1.0):
            p = np.zeros((a.size, 3))
            p[:, ax] = side
            p[:, o1] = a
            p[:, o2] = b
            pts.append(p)
    return np.asarray(centre) + np.concatenate(pts) * np.asarray(half)


def psi_t(mu, t0, tau, tgrid):
    """Lemma 3 by sampling: pi inside the cuboid, else the largest sampled angle."""
    if np.all(np.abs(mu - t0) <= tau):
        return math.pi
    return float(angle(mu[None, :] - tgrid, (mu - t0)[None, :]).max())


def psi_r_inverse(p, r0, rgrid):
    """Lemma 2 by sampling, for the inverse rotation that eq. 25 applies to p:
    the largest angle between R_r^{-1} p and R_r0^{-1} p over the surface
    samples r, capped at pi."""
    Rs = Rotation.from_rotvec(rgrid).as_matrix()          # (n, 3, 3)
    R0 = Rotation.from_rotvec(r0).as_matrix()
    q = np.einsum("nji,j->ni", Rs, p)                      # R_r^T p
    q0 = R0.T @ p
    return min(float(angle(q, q0[None, :]).max()), math.pi)


def objective_terms(scene, r, t):
    """S11(t) and S12(R_r, t) of Lemma 1 (eqs. 10-13), class-weighted."""
    w1, w2, l1, l2, phil = class_weights(scene)
    d = scene.mu - t
    rho = np.linalg.norm(d, axis=1)
    u = d / rho[:, None]
    kap = (rho / scene.sigma) ** 2 + 1.0
    R = Rotation.from_rotvec(r).as_matrix()
    same11 = l1[:, None] == l1[None, :]
    s11 = np.sum(same11 * w1[:, None] * w1[None, :] *
                 np.exp(log_ratio(kap[:, None], kap[None, :], angle(u[:, None, :], u[None, :, :]))))
    ru = u @ R.T
    same12 = l1[:, None] == l2[None, :]
    s12 = np.sum(same12 * w1[:, None] * w2[None, :] *
                 np.exp(log_ratio(kap[:, None], scene.kappa2[None, :], angle(ru[:, None, :], scene.dir2[None, :, :]))))
    return phil * s11, phil * s12


def lower_bound(scene, r0, hr, t0, tau, n_t=9, n_r=13, diagonal="literal"):
    """Eq. 21 for the cube centred at (r0, t0) with half-widths (hr, tau), by
    sampling.  diagonal="literal" takes A = min(pi, 2 psi_t) for i = j as
    eq. 24 gives it; diagonal="zero" takes the exact angle 0 between
    mu_1i - t and itself.  Returns a dict with S11_lo, S12_hi, lb and the
    sampled angles, or None when no sampled translation of the cube is
    feasible."""
    r0, hr, t0, tau = (np.asarray(v, float) for v in (r0, hr, t0, tau))
    w1, w2, l1, l2, phil = class_weights(scene)
    M, N = scene.M, scene.N
    tg = box_grid(t0, tau, n_t)
    dist = np.linalg.norm(scene.mu[None, :, :] - tg[:, None, :], axis=2)     # (nt, M)
    feas = np.all(dist >= scene.zeta, axis=1)
    if not feas.any():
        return None
    kap_t = (dist[feas] / scene.sigma[None, :]) ** 2 + 1.0                  # (nf, M)
    pt = np.array([psi_t(scene.mu[i], t0, tau, tg) for i in range(M)])
    rg = surface_grid(r0, hr, n_r)
    pr = np.array([psi_r_inverse(scene.dir2[j], r0, rg) for j in range(N)])
    c = scene.mu - t0
    R0 = Rotation.from_rotvec(r0).as_matrix()
    rinv_mu = scene.dir2 @ R0                                               # rows R0^T mu_2j
    A = np.minimum(math.pi, angle(c[:, None, :], c[None, :, :]) + pt[:, None] + pt[None, :])
    if diagonal == "zero":
        A[np.arange(M), np.arange(M)] = 0.0
    B = np.maximum(0.0, angle(c[:, None, :], rinv_mu[None, :, :]) - pt[:, None] - pr[None, :])
    s11 = 0.0
    for i in range(M):
        for k in range(M):
            if l1[i] != l1[k]:
                continue
            v = np.exp(log_ratio(kap_t[:, i], kap_t[:, k], A[i, k])).min()
            s11 += w1[i] * w1[k] * v
    s12 = 0.0
    for i in range(M):
        for j in range(N):
            if l1[i] != l2[j]:
                continue
            v = np.exp(log_ratio(kap_t[:, i], scene.kappa2[j], B[i, j])).max()
            s12 += w1[i] * w2[j] * v
    return {"S11_lo": phil * s11, "S12_hi": phil * s12, "lb": phil * (s11 - 2.0 * s12),
            "psi_t": pt, "psi_r": pr}
