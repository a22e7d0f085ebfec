"""ctypes wrapper of the FP64 CPU oracle (oracle/gosma_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "gosma_oracle.c"
SRC_MIXGEN = HERE / "mixgen_oracle.c"
LIB = HERE / "libgosma_oracle.so"


def build(force=True):
    """Compile the oracle (gcc, -O2, OpenMP).  No fast-math: plain IEEE FP64."""
    if LIB.exists() and not force:
        return LIB
    tmp = LIB.with_suffix(".so.tmp")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           "-D_POSIX_C_SOURCE=200809L", str(SRC), str(SRC_MIXGEN), "-o", str(tmp), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class Problem(C.Structure):
    _fields_ = [("M", C.c_int), ("N", C.c_int), ("n_labels", C.c_int),
                ("mu", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)),
                ("phi1", C.POINTER(C.c_double)), ("label1", C.POINTER(C.c_int32)),
                ("dir2", C.POINTER(C.c_double)), ("kappa2", C.POINTER(C.c_double)),
                ("phi2", C.POINTER(C.c_double)), ("label2", C.POINTER(C.c_int32))]


class Domain(C.Structure):
    _fields_ = [("r_lo", C.c_double * 3), ("r_hi", C.c_double * 3), ("t_lo", C.c_double * 3),
                ("t_hi", C.c_double * 3), ("zeta", C.c_double)]


class Bound(C.Structure):
    _fields_ = [("ub", C.c_double), ("lb", C.c_double), ("s11_ub", C.c_double), ("s12_ub", C.c_double),
                ("s11_lo", C.c_double), ("s12_hi", C.c_double), ("psi_r", C.c_double),
                ("psi_t_mean", C.c_double), ("status", C.c_int32), ("split_rot", C.c_int32),
                ("top8", C.c_double * 8)]


class Opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("batch_parents", C.c_int64), ("max_iters", C.c_int64),
                ("time_limit_s", C.c_double), ("nthreads", C.c_int), ("sma_iters", C.c_int)]


class SmaOpts(C.Structure):
    _fields_ = [("max_iters", C.c_int), ("memory", C.c_int), ("gtol", C.c_double), ("ftol", C.c_double)]


class Result(C.Structure):
    _fields_ = [("f_best", C.c_double), ("lb_global", C.c_double), ("f_norm_best", C.c_double),
                ("lb_norm", C.c_double), ("S22", C.c_double), ("r", C.c_double * 3),
                ("t", C.c_double * 3), ("iters", C.c_int64), ("cubes", C.c_int64),
                ("max_queue", C.c_int64), ("status", C.c_int32), ("seconds", C.c_double),
                ("sma_runs", C.c_int64), ("sma_improved", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB.exists():
            build()
        L = C.CDLL(str(LIB))
        d3 = C.POINTER(C.c_double)
        L.oracle_log_Z.restype = C.c_double
        L.oracle_log_Z.argtypes = [C.c_double]
        L.oracle_vmf_pdf.restype = C.c_double
        L.oracle_vmf_pdf.argtypes = [d3, d3, C.c_double]
        L.oracle_pn_pdf.restype = C.c_double
        L.oracle_pn_pdf.argtypes = [d3, d3, C.c_double]
        L.oracle_qpn_kappa.restype = C.c_double
        L.oracle_qpn_kappa.argtypes = [d3, C.c_double]
        L.oracle_rodrigues.argtypes = [d3, d3]
        L.oracle_objective.restype = C.c_double
        L.oracle_objective.argtypes = [C.POINTER(Problem), d3, d3, d3, d3]
        L.oracle_S22.restype = C.c_double
        L.oracle_S22.argtypes = [C.POINTER(Problem)]
        L.oracle_psi_t.restype = C.c_double
        L.oracle_psi_t.argtypes = [d3, d3, d3]
        L.oracle_psi_r.restype = C.c_double
        L.oracle_psi_r.argtypes = [d3]
        L.oracle_psi_r_dir.restype = C.c_double
        L.oracle_psi_r_dir.argtypes = [d3, d3, d3, C.c_double]
        L.oracle_left_jacobian.restype = None
        L.oracle_left_jacobian.argtypes = [d3, d3]
        L.oracle_s11_lower_log.restype = C.c_double
        L.oracle_s11_lower_log.argtypes = [C.c_double] * 5
        L.oracle_s12_upper_term.restype = C.c_double
        L.oracle_s12_upper_term.argtypes = [C.c_double] * 4
        L.oracle_s12_upper_term_pieces.restype = C.c_double
        L.oracle_s12_upper_term_pieces.argtypes = [C.c_double] * 4 + [C.c_int]
        L.oracle_s12_expansion_log.restype = C.c_double
        L.oracle_s12_expansion_log.argtypes = [C.c_double] * 4
        L.oracle_set_kappa_pieces.restype = C.c_int
        L.oracle_set_kappa_pieces.argtypes = [C.c_int]
        L.oracle_decode.argtypes = [C.c_uint64, d3, d3, d3, d3]
        L.oracle_eval_bounds.argtypes = [C.POINTER(Problem), C.POINTER(Domain), C.POINTER(C.c_uint64),
                                         C.POINTER(C.c_uint64), C.c_int64, C.POINTER(Bound), C.c_int]
        L.oracle_solve.argtypes = [C.POINTER(Problem), C.POINTER(Domain), C.POINTER(Opts), C.POINTER(Result)]
        L.oracle_objective_grad.restype = C.c_double
        L.oracle_objective_grad.argtypes = [C.POINTER(Problem), d3, d3, d3]
        i32p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        for name in ("oracle_dpmeans", "oracle_dpvmf_means"):
            getattr(L, name).restype = C.c_int
            getattr(L, name).argtypes = [d3, C.c_int64, C.c_double, C.c_int, C.c_int, i32p, d3, i64p,
                                         C.POINTER(C.c_int)]
        L.oracle_vmf_kappa_ml.restype = C.c_double
        L.oracle_vmf_kappa_ml.argtypes = [C.c_double]
        L.oracle_gmm_sigma_ml.restype = None
        L.oracle_gmm_sigma_ml.argtypes = [d3, C.c_int64, i32p, d3, i64p, C.c_int, d3]
        L.oracle_sma.restype = C.c_int
        L.oracle_sma.argtypes = [C.POINTER(Problem), C.POINTER(Domain), d3, d3, C.POINTER(SmaOpts), d3, d3, d3]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleProblem:
    """Holds contiguous FP64 copies of a scene and the ctypes structs."""

    def __init__(self, scene):
        self.mu = np.ascontiguousarray(scene.mu, dtype=np.float64)
        self.sigma = np.ascontiguousarray(scene.sigma, dtype=np.float64)
        self.phi1 = np.ascontiguousarray(scene.phi1, dtype=np.float64)
        self.dir2 = np.ascontiguousarray(scene.dir2, dtype=np.float64)
        self.kappa2 = np.ascontiguousarray(scene.kappa2, dtype=np.float64)
        self.phi2 = np.ascontiguousarray(scene.phi2, dtype=np.float64)
        self.label1 = None if scene.label1 is None else np.ascontiguousarray(scene.label1, dtype=np.int32)
        self.label2 = None if scene.label2 is None else np.ascontiguousarray(scene.label2, dtype=np.int32)
        ip = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))
        self.p = Problem(self.mu.shape[0], self.dir2.shape[0], scene.n_labels if self.label1 is not None else 1,
                         _dp(self.mu), _dp(self.sigma), _dp(self.phi1), ip(self.label1),
                         _dp(self.dir2), _dp(self.kappa2), _dp(self.phi2), ip(self.label2))
        self.d = Domain((C.c_double * 3)(*scene.r_lo), (C.c_double * 3)(*scene.r_hi),
                        (C.c_double * 3)(*scene.t_lo), (C.c_double * 3)(*scene.t_hi), float(scene.zeta))

    def objective(self, r, t):
        r = np.ascontiguousarray(r, dtype=np.float64)
        t = np.ascontiguousarray(t, dtype=np.float64)
        s11 = C.c_double()
        s12 = C.c_double()
        f = lib().oracle_objective(C.byref(self.p), _dp(r), _dp(t), C.byref(s11), C.byref(s12))
        return f, s11.value, s12.value

    def S22(self):
        return lib().oracle_S22(C.byref(self.p))

    def bounds(self, rkeys, tkeys, nthreads=0):
        rk = np.ascontiguousarray(rkeys, dtype=np.uint64)
        tk = np.ascontiguousarray(tkeys, dtype=np.uint64)
        n = rk.shape[0]
        out = (Bound * max(n, 1))()
        lib().oracle_eval_bounds(C.byref(self.p), C.byref(self.d), rk.ctypes.data_as(C.POINTER(C.c_uint64)),
                                 tk.ctypes.data_as(C.POINTER(C.c_uint64)), n, out, nthreads)
        arr = np.ctypeslib.as_array(out)[:n]
        return {name: np.array(arr[name]) for name in arr.dtype.names}

    def objective_grad(self, r, t):
        """Objective and its gradient (6,) with respect to (r, t)."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        t = np.ascontiguousarray(t, dtype=np.float64)
        g = np.zeros(6)
        f = lib().oracle_objective_grad(C.byref(self.p), _dp(r), _dp(t), _dp(g))
        return f, g

    def sma(self, r0, t0, max_iters=100, memory=5, gtol=1e-6, ftol=1e-9):
        """SMA (L-BFGS) from (r0, t0): {r, t, f, iters} (iters -1: start not allowed)."""
        r0 = np.ascontiguousarray(r0, dtype=np.float64)
        t0 = np.ascontiguousarray(t0, dtype=np.float64)
        r, t, f = np.zeros(3), np.zeros(3), np.zeros(1)
        o = SmaOpts(max_iters, memory, gtol, ftol)
        it = lib().oracle_sma(C.byref(self.p), C.byref(self.d), _dp(r0), _dp(t0), C.byref(o), _dp(r), _dp(t), _dp(f))
        return {"r": r, "t": t, "f": float(f[0]), "iters": it}

    def solve(self, eps, batch_parents, max_iters=0, time_limit_s=0.0, nthreads=0, sma_iters=0):
        o = Opts(eps, batch_parents, max_iters, time_limit_s, nthreads, sma_iters)
        res = Result()
        lib().oracle_solve(C.byref(self.p), C.byref(self.d), C.byref(o), C.byref(res))
        return {name: (list(getattr(res, name)) if name in ("r", "t") else getattr(res, name))
                for name, _ in Result._fields_}


def log_Z(x):
    return lib().oracle_log_Z(float(x))


def vmf_pdf(f, mu_hat, kappa):
    f = np.ascontiguousarray(f, dtype=np.float64)
    m = np.ascontiguousarray(mu_hat, dtype=np.float64)
    return lib().oracle_vmf_pdf(_dp(f), _dp(m), float(kappa))


def pn_pdf(f, mu, sigma2):
    f = np.ascontiguousarray(f, dtype=np.float64)
    m = np.ascontiguousarray(mu, dtype=np.float64)
    return lib().oracle_pn_pdf(_dp(f), _dp(m), float(sigma2))


def qpn_kappa(mu, sigma):
    m = np.ascontiguousarray(mu, dtype=np.float64)
    return lib().oracle_qpn_kappa(_dp(m), float(sigma))


def rodrigues(r):
    r = np.ascontiguousarray(r, dtype=np.float64)
    R = np.zeros(9)
    lib().oracle_rodrigues(_dp(r), _dp(R))
    return R.reshape(3, 3)


def psi_t(p, t0, tau):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (p, t0, tau)]
    return lib().oracle_psi_t(_dp(a[0]), _dp(a[1]), _dp(a[2]))


def psi_r(half):
    h = np.ascontiguousarray(half, dtype=np.float64)
    return lib().oracle_psi_r(_dp(h))


def psi_r_dir(r0, half, w, psit):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (r0, half, w)]
    return lib().oracle_psi_r_dir(_dp(a[0]), _dp(a[1]), _dp(a[2]), float(psit))


def left_jacobian(r):
    J = np.zeros(9)
    lib().oracle_left_jacobian(_dp(np.ascontiguousarray(r, dtype=np.float64)), _dp(J))
    return J.reshape(3, 3)


def s11_lower_log(alo, ahi, blo, bhi, A):
    return lib().oracle_s11_lower_log(alo, ahi, blo, bhi, A)


def s12_upper_term(alo, ahi, b, B):
    return lib().oracle_s12_upper_term(alo, ahi, b, B)


def s12_upper_term_pieces(alo, ahi, b, B, m):
    return lib().oracle_s12_upper_term_pieces(alo, ahi, b, B, int(m))


def s12_expansion_log(e0, e1, b, B):
    return lib().oracle_s12_expansion_log(e0, e1, b, B)


def set_kappa_pieces(m):
    """Pieces of the kappa interval of the S12 upper term in every later cube
    bound of the oracle (1 to 64; 1 is the default reading)."""
    if lib().oracle_set_kappa_pieces(int(m)) != 0:
        raise ValueError("kappa pieces must be in 1..64")


def decode(key, lo, hi):
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    c = np.zeros(3)
    h = np.zeros(3)
    lib().oracle_decode(C.c_uint64(int(key)), _dp(lo), _dp(hi), _dp(c), _dp(h))
    return c, h


def _cluster(fn, x, lam, max_clusters, max_passes):
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    z = np.zeros(max(n, 1), dtype=np.int32)
    mu = np.zeros((max_clusters, 3))
    cnt = np.zeros(max_clusters, dtype=np.int64)
    passes = C.c_int()
    K = fn(_dp(x), n, float(lam), int(max_clusters), int(max_passes), z.ctypes.data_as(C.POINTER(C.c_int32)),
           _dp(mu), cnt.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(passes))
    return {"K": K, "labels": z[:n], "centres": mu[:K].copy(), "counts": cnt[:K].copy(), "passes": passes.value}


def dpmeans(x, lam, max_clusters=1024, max_passes=100):
    """DP-means (serial batch algorithm): {K, labels, centres, counts, passes}."""
    return _cluster(lib().oracle_dpmeans, x, lam, max_clusters, max_passes)


def dpvmf_means(x, cos_lam, max_clusters=1024, max_passes=100):
    """DP-vMF-means on unit vectors: {K, labels, centres (unit), counts, passes}."""
    return _cluster(lib().oracle_dpvmf_means, x, cos_lam, max_clusters, max_passes)


def vmf_kappa_ml(rbar):
    return lib().oracle_vmf_kappa_ml(float(rbar))


def gmm_sigma_ml(x, labels, centres, counts):
    x = np.ascontiguousarray(x, dtype=np.float64)
    z = np.ascontiguousarray(labels, dtype=np.int32)
    mu = np.ascontiguousarray(centres, dtype=np.float64)
    cnt = np.ascontiguousarray(counts, dtype=np.int64)
    K = mu.shape[0]
    s = np.zeros(max(K, 1))
    lib().oracle_gmm_sigma_ml(_dp(x), x.shape[0], z.ctypes.data_as(C.POINTER(C.c_int32)), _dp(mu),
                              cnt.ctypes.data_as(C.POINTER(C.c_int64)), K, _dp(s))
    return s[:K]
