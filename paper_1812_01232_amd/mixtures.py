"""Mixture generation (Section 7): a GMM from a 3D point set and a vMF
mixture from bearing vectors, both clustered and fitted by the library
(gosma_dpmeans, gosma_dpvmf_means).  This module only selects the points of
each class and gathers the per-class results; the weights are the cluster
sizes, which gosma_set_mixtures normalises.
"""
from __future__ import annotations

import numpy as np


def mixtures_from_data(ctx, points, bearings, lam_points, cos_lam_bearings, labels_points=None,
                       labels_bearings=None, n_labels=1, max_clusters=1024, max_passes=100, sigma_min=1e-3,
                       kappa_max=1e5):
    """{mu, sigma, phi1, dir2, kappa2, phi2[, label1, label2, n_labels]} for
    Context.set_scene-style use.  With labels, each class is clustered on its
    own (semantic mixtures, eq. 17)."""
    points = np.asarray(points, dtype=np.float64)
    bearings = np.asarray(bearings, dtype=np.float64)
    classes = range(n_labels) if labels_points is not None else [None]
    out = {k: [] for k in ("mu", "sigma", "phi1", "dir2", "kappa2", "phi2", "label1", "label2")}
    for c in classes:
        P = points if c is None else points[np.asarray(labels_points) == c]
        B = bearings if c is None else bearings[np.asarray(labels_bearings) == c]
        if len(P) == 0 or len(B) == 0:
            continue
        g = ctx.dpmeans(P, lam_points, max_clusters=max_clusters, max_passes=max_passes, sigma_min=sigma_min)
        v = ctx.dpvmf_means(B, cos_lam_bearings, max_clusters=max_clusters, max_passes=max_passes,
                            kappa_max=kappa_max)
        out["mu"].append(g["centres"])
        out["sigma"].append(g["spread"])
        out["phi1"].append(g["counts"].astype(np.float64))
        out["dir2"].append(v["centres"])
        out["kappa2"].append(v["spread"])
        out["phi2"].append(v["counts"].astype(np.float64))
        out["label1"].append(np.full(g["K"], 0 if c is None else c, dtype=np.int32))
        out["label2"].append(np.full(v["K"], 0 if c is None else c, dtype=np.int32))
    res = {k: np.concatenate(v) for k, v in out.items()}
    if labels_points is None:
        res.pop("label1")
        res.pop("label2")
    else:
        res["n_labels"] = n_labels
    return res
