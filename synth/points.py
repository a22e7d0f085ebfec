"""Seeded synthetic point sets and bearing vectors, the inputs of the mixture
generation step (Section 7 clusters a 3D point set and an image's bearing
vectors into the two mixtures).

The paper's point clouds and panoramas (Stanford 2D-3D-S) are not available;
these stand in for them: points drawn from a scene's Gaussian mixture (the
geometry the mixtures are meant to summarise), and bearing vectors of a
random subset of them seen from the true pose, with angular noise and
outlier directions.  Every coordinate is rounded to a binary grid (points to
2^-24 m, directions to 2^-30), so that sums of up to 2^20 of them are exact in
FP64 whatever the order of addition.  Nothing here implements the clustering
or the fits.
"""
from __future__ import annotations

import math

import numpy as np

from .scenes import _angular_noise, _uniform_sphere

POINT_GRID = 2.0 ** -24
DIR_GRID = 2.0 ** -30


def quantize(x, grid):
    return np.round(np.asarray(x, dtype=np.float64) / grid) * grid


def point_cloud(scene, n, seed):
    """n points from the scene's Gaussian mixture (component by weight), with
    the component each came from."""
    rng = np.random.default_rng(seed)
    comp = rng.choice(scene.M, size=n, p=scene.phi1 / scene.phi1.sum())
    pts = scene.mu[comp] + rng.normal(size=(n, 3)) * scene.sigma[comp][:, None]
    return quantize(pts, POINT_GRID), comp


def bearings(scene, points, n, seed, noise_deg=1.0, outlier_frac=0.3):
    """n bearing vectors: (1 - outlier_frac) n camera-frame directions
    R (x - t) / |x - t| of random points (angular noise of noise_deg), the
    rest uniform on the sphere; returns (directions, is_inlier)."""
    rng = np.random.default_rng(seed)
    n_in = int(round((1.0 - outlier_frac) * n))
    pick = rng.choice(points.shape[0], size=n_in, replace=n_in > points.shape[0])
    d = (points[pick] - scene.t_gt) @ scene.R_gt.T
    d /= np.linalg.norm(d, axis=1)[:, None]
    d = _angular_noise(rng, d, math.radians(noise_deg))
    out = _uniform_sphere(rng, n - n_in)
    dirs = np.concatenate([d, out])
    inl = np.concatenate([np.ones(n_in, bool), np.zeros(n - n_in, bool)])
    perm = rng.permutation(n)
    return quantize(dirs[perm], DIR_GRID), inl[perm]


def blobs(n_blobs, per_blob, spread, radius, seed, dim_scale=(1.0, 1.0, 1.0)):
    """Well-separated blobs for clustering checks: centres on a grid `spread`
    apart, points uniform in a ball of `radius` around them."""
    rng = np.random.default_rng(seed)
    k = math.ceil(n_blobs ** (1 / 3))
    grid = np.array([(i, j, l) for i in range(k) for j in range(k) for l in range(k)], dtype=np.float64)[:n_blobs]
    centres = grid * spread * np.asarray(dim_scale)
    v = rng.normal(size=(n_blobs * per_blob, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    r = radius * rng.uniform(size=(n_blobs * per_blob, 1)) ** (1 / 3)
    lab = np.repeat(np.arange(n_blobs), per_blob)
    pts = centres[lab] + v * r
    perm = rng.permutation(len(lab))
    return quantize(pts[perm], POINT_GRID), lab[perm]


def direction_blobs(n_blobs, per_blob, max_angle_deg, seed):
    """Directions around n_blobs well-separated unit axes (spread at most
    max_angle_deg around each)."""
    rng = np.random.default_rng(seed)
    axes = []
    while len(axes) < n_blobs:
        a = _uniform_sphere(rng, 1)[0]
        if all(np.dot(a, b) < math.cos(math.radians(40)) for b in axes):
            axes.append(a)
    axes = np.array(axes)
    lab = np.repeat(np.arange(n_blobs), per_blob)
    d = _angular_noise(rng, axes[lab], math.radians(max_angle_deg) / 3)
    perm = rng.permutation(len(lab))
    return quantize(d[perm], DIR_GRID), lab[perm]
