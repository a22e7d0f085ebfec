"""Seeded synthetic GMM / vMF-mixture scenes and random sub-cube sets.

This module is the only code shared by the CPU oracle and the HIP path: it
draws random inputs and nothing else.  It holds none of the bound or
objective arithmetic; the one formula it applies is the input recipe of the
scenes themselves -- an image vMF component is the projection of a 3D Gaussian
through the ground-truth pose with concentration (depth / sigma)^2 + 1, the
qPN map of Section 3 (eq. 6) that the workloads are defined by.  The
ground-truth rotation is drawn as a unit quaternion and turned into a matrix
with the quaternion formula (not the angle-axis formula the method uses), so
a test that evaluates the objective at the stored pose cross-checks the two.

Workloads (all FP64, seed = 1000 * config + scene index, PCG64):

* ``cfg1``: 16 Gaussians, means uniform in [-2,2]x[-2,2]x[-1,1] m, sigma 0.1 m,
  equal weights; 16 noise-free projected vMF components; translation domain
  [-0.5,0.5]^3 m.
* ``cfg2``: 64 Gaussians, means uniform in a 10 x 10 x 3 m room, sigma
  U[0.05, 0.3] m, Dirichlet(1) weights; 45 projected inliers with 1 degree
  angular noise plus 19 outlier directions uniform on the sphere; translation
  domain [-1,1]^3 m.
* ``cfg3``: 256 x 256 components in the cfg2 room, labels uniform over 8
  classes, 30 % outliers, kappa clipped to [50, 2000].
* ``batch``: many cfg2-style problems with M, N drawn from [16, 256].

Every scene keeps all Gaussian means at least zeta + 0.05 m from the
ground-truth camera centre (resampled), so the ground truth is feasible.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Octree key layout shared by both sides of the boundary (documented in
# include/gosma.h): bits 0-18 z index, 19-37 y index, 38-56 x index,
# 57-62 level.  Level L splits each axis of the root box into 2^L cells.
KEY_BITS = 19
MAX_LEVEL = 19


def pack_key(level, ix, iy, iz):
    level = np.asarray(level, dtype=np.uint64)
    ix = np.asarray(ix, dtype=np.uint64)
    iy = np.asarray(iy, dtype=np.uint64)
    iz = np.asarray(iz, dtype=np.uint64)
    return (level << np.uint64(57)) | (ix << np.uint64(38)) | (iy << np.uint64(19)) | iz


def unpack_key(key):
    key = np.asarray(key, dtype=np.uint64)
    m = np.uint64((1 << KEY_BITS) - 1)
    return ((key >> np.uint64(57)) & np.uint64(63), (key >> np.uint64(38)) & m,
            (key >> np.uint64(19)) & m, key & m)


@dataclass
class Scene:
    """One pose problem: a GMM (theta_1), a vMF mixture (theta_2), a domain."""
    mu: np.ndarray            # (M, 3) Gaussian means, metres
    sigma: np.ndarray         # (M,) isotropic standard deviations
    phi1: np.ndarray          # (M,) weights, sum 1
    dir2: np.ndarray          # (N, 3) unit mean directions
    kappa2: np.ndarray        # (N,) concentrations
    phi2: np.ndarray          # (N,) weights, sum 1
    r_gt: np.ndarray          # (3,) ground-truth angle-axis rotation, |r| <= pi
    R_gt: np.ndarray          # (3, 3) the same rotation as a matrix
    t_gt: np.ndarray          # (3,) ground-truth camera centre
    t_lo: np.ndarray          # (3,) translation domain box
    t_hi: np.ndarray
    r_lo: np.ndarray = field(default_factory=lambda: np.full(3, -math.pi))
    r_hi: np.ndarray = field(default_factory=lambda: np.full(3, math.pi))
    zeta: float = 0.5
    eps: float = 1e-3
    label1: Optional[np.ndarray] = None   # (M,) int32 class labels or None
    label2: Optional[np.ndarray] = None   # (N,) int32
    n_labels: int = 1
    inlier_src: Optional[np.ndarray] = None  # (N,) source Gaussian of each vMF, -1 for outliers
    name: str = ""

    @property
    def M(self):
        return int(self.mu.shape[0])

    @property
    def N(self):
        return int(self.dir2.shape[0])


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def random_rotation(rng):
    """Uniform rotation: normalised Gaussian quaternion -> (matrix, angle-axis)."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    if q[0] < 0:                      # w >= 0 gives rotation angle <= pi
        q = -q
    w, x, y, z = q
    R = np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])
    s = math.sqrt(x * x + y * y + z * z)
    angle = 2.0 * math.atan2(s, w)
    r = np.zeros(3) if s == 0 else np.array([x, y, z]) / s * angle
    return R, r


def _means_clear_of(rng, n, lo, hi, t, clearance):
    mu = rng.uniform(lo, hi, size=(n, 3))
    for _ in range(1000):
        bad = np.linalg.norm(mu - t, axis=1) < clearance
        if not bad.any():
            return mu
        mu[bad] = rng.uniform(lo, hi, size=(int(bad.sum()), 3))
    raise RuntimeError("could not place Gaussian means clear of the camera")


def _uniform_sphere(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _angular_noise(rng, u, sigma_rad):
    """Isotropic tangent-plane Gaussian perturbation of unit vectors."""
    if sigma_rad <= 0:
        return u.copy()
    n = rng.standard_normal(u.shape) * sigma_rad
    n -= np.sum(n * u, axis=1, keepdims=True) * u
    v = u + n
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _project(mu, sigma, R, t):
    """Camera-frame bearings R (mu - t) / |mu - t| and concentrations (|mu - t|/sigma)^2 + 1."""
    d = (mu - t) @ R.T
    depth = np.linalg.norm(d, axis=1)
    return d / depth[:, None], (depth / sigma) ** 2 + 1.0


def make_scene(M, N, n_inliers, *, seed, room_lo, room_hi, t_half, sigma_range,
               dirichlet, noise_deg, n_labels=1, kappa_clip=None, outlier_kappa=None,
               zeta=0.5, eps=1e-3, name=""):
    rng = _rng(seed)
    R, r = random_rotation(rng)
    t = rng.uniform(-t_half, t_half, size=3)
    mu = _means_clear_of(rng, M, np.asarray(room_lo, float), np.asarray(room_hi, float), t, zeta + 0.05)
    if sigma_range[0] == sigma_range[1]:
        sigma = np.full(M, float(sigma_range[0]))
    else:
        sigma = rng.uniform(sigma_range[0], sigma_range[1], size=M)
    phi1 = rng.dirichlet(np.ones(M)) if dirichlet else np.full(M, 1.0 / M)
    label1 = rng.integers(0, n_labels, size=M).astype(np.int32) if n_labels > 1 else None

    n_in = min(n_inliers, M, N)
    src = rng.choice(M, size=n_in, replace=False) if n_in < M else rng.permutation(M)[:n_in]
    dirs, kap = _project(mu[src], sigma[src], R, t)
    dirs = _angular_noise(rng, dirs, math.radians(noise_deg))
    if kappa_clip is not None:
        kap = np.clip(kap, kappa_clip[0], kappa_clip[1])
    phi2_in = phi1[src].copy()
    n_out = N - n_in
    out_dirs = _uniform_sphere(rng, n_out)
    if outlier_kappa is not None:
        out_kap = rng.uniform(outlier_kappa[0], outlier_kappa[1], size=n_out)
    else:
        out_kap = rng.choice(kap, size=n_out, replace=True) if n_out else np.zeros(0)
    dir2 = np.concatenate([dirs, out_dirs])
    kappa2 = np.concatenate([kap, out_kap])
    phi2 = np.concatenate([phi2_in, np.full(n_out, 1.0 / N)])
    phi2 /= phi2.sum()
    label2 = None
    if label1 is not None:
        label2 = np.concatenate([label1[src], rng.integers(0, n_labels, size=n_out)]).astype(np.int32)
    inlier_src = np.concatenate([src, -np.ones(n_out, dtype=np.int64)])
    return Scene(mu=mu, sigma=sigma, phi1=phi1, dir2=dir2, kappa2=kappa2, phi2=phi2,
                 r_gt=r, R_gt=R, t_gt=t, t_lo=np.full(3, -t_half), t_hi=np.full(3, t_half),
                 zeta=zeta, eps=eps, label1=label1, label2=label2, n_labels=n_labels,
                 inlier_src=inlier_src, name=name)


def cfg1_scene(idx=0):
    """16 x 16, noise-free, 4 x 4 x 2 m box, sigma 0.1 m, equal weights."""
    return make_scene(16, 16, 16, seed=1000 * 1 + idx, room_lo=(-2, -2, -1), room_hi=(2, 2, 1),
                      t_half=0.5, sigma_range=(0.1, 0.1), dirichlet=False, noise_deg=0.0,
                      name=f"cfg1-{idx}")


def cfg2_scene(idx=0, seed=None):
    """64 x 64: 45 noisy inliers + 19 outliers, 10 x 10 x 3 m room."""
    s = 1000 * 2 + idx if seed is None else seed
    return make_scene(64, 64, 45, seed=s, room_lo=(-5, -5, -1.5), room_hi=(5, 5, 1.5),
                      t_half=1.0, sigma_range=(0.05, 0.3), dirichlet=True, noise_deg=1.0,
                      name=f"cfg2-{idx}")


def cfg3_scene(idx=0):
    """256 x 256, 8 labels, 30 % outliers, kappa in [50, 2000]."""
    return make_scene(256, 256, int(round(0.7 * 256)), seed=1000 * 3 + idx, room_lo=(-5, -5, -1.5),
                      room_hi=(5, 5, 1.5), t_half=1.0, sigma_range=(0.05, 0.3), dirichlet=True,
                      noise_deg=1.0, n_labels=8, kappa_clip=(50.0, 2000.0),
                      outlier_kappa=(50.0, 2000.0), name=f"cfg3-{idx}")


def small_scene(M, N, seed, noise_deg=0.0, n_inliers=None, sigma=(0.1, 0.1), t_half=0.5,
                room=((-2, -2, -1), (2, 2, 1)), n_labels=1):
    """Small scenes for brute-force checks."""
    return make_scene(M, N, N if n_inliers is None else n_inliers, seed=seed, room_lo=room[0],
                      room_hi=room[1], t_half=t_half, sigma_range=sigma, dirichlet=True,
                      noise_deg=noise_deg, n_labels=n_labels, name=f"small-{M}x{N}-{seed}")


def batch_scenes(n_problems=128, seed=4000, lo=16, hi=256):
    """Independent cfg2-style problems with M, N uniform on [lo, hi]."""
    rng = _rng(seed)
    Ms = rng.integers(lo, hi + 1, size=n_problems)
    Ns = rng.integers(lo, hi + 1, size=n_problems)
    out = []
    for p in range(n_problems):
        M, N = int(Ms[p]), int(Ns[p])
        out.append(make_scene(M, N, int(round(45 / 64 * N)), seed=seed * 10 + p, room_lo=(-5, -5, -1.5),
                              room_hi=(5, 5, 1.5), t_half=1.0, sigma_range=(0.05, 0.3),
                              dirichlet=True, noise_deg=1.0, name=f"batch-{p}"))
    return out


def random_cubes(scene, n, seed, r_levels=(1, 8), t_levels=(0, 8)):
    """Random sub-cubes: levels uniform on the given ranges, indices uniform on
    the level grid; rotation cubes lying wholly outside the radius-pi ball of
    angle-axis vectors are redrawn (they contain no rotation)."""
    rng = _rng(seed)
    rk = np.empty(n, np.uint64)
    tk = np.empty(n, np.uint64)
    r_lo, r_hi = np.asarray(scene.r_lo, float), np.asarray(scene.r_hi, float)
    filled = 0
    while filled < n:
        m = 2 * (n - filled) + 16
        lr = rng.integers(r_levels[0], r_levels[1] + 1, size=m)
        lt = rng.integers(t_levels[0], t_levels[1] + 1, size=m)
        ir = np.stack([rng.integers(0, 1 << l, size=3) for l in lr]) if m else np.zeros((0, 3), int)
        it = np.stack([rng.integers(0, 1 << l, size=3) for l in lt]) if m else np.zeros((0, 3), int)
        w = (r_hi - r_lo)[None, :] / (2.0 ** lr)[:, None]
        lo = r_lo[None, :] + ir * w
        hi = lo + w
        nearest = np.clip(0.0, lo, hi)
        ok = np.linalg.norm(nearest, axis=1) <= math.pi
        idx = np.nonzero(ok)[0][: n - filled]
        k = len(idx)
        rk[filled:filled + k] = pack_key(lr[idx], ir[idx, 0], ir[idx, 1], ir[idx, 2])
        tk[filled:filled + k] = pack_key(lt[idx], it[idx, 0], it[idx, 1], it[idx, 2])
        filled += k
    return rk, tk


def cube_geometry(key, lo, hi):
    """Centre and half-widths of an octree cell of the box [lo, hi] (for tests)."""
    L, ix, iy, iz = (np.asarray(v, dtype=np.int64) for v in unpack_key(key))
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    half = (hi - lo)[None, :] / (2.0 ** (L + 1))[..., None]
    idx = np.stack([ix, iy, iz], axis=-1)
    return lo + (2 * idx + 1) * half, half
