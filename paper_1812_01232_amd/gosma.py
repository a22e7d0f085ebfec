"""Python binding of libgosma (ctypes).

Argument marshalling only: every step of the bound evaluation and of the
branch-and-bound runs in the HIP library.  Device buffers are torch tensors
on a ROCm device; their data pointers and the current HIP stream are passed
through the C-ABI of include/gosma.h.  The library must have been built
(python -m paper_1812_01232_amd.build); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "libgosma.so"

GOSMA_OK = 0
QUEUE_OVERFLOW = -4
ERRORS = {-1: "GOSMA_E_INVAL", -2: "GOSMA_E_NOMEM", -3: "GOSMA_E_HIP", -4: "GOSMA_E_QUEUE_OVERFLOW",
          -5: "GOSMA_E_STATE"}
FLAG_SPLIT_ROT, FLAG_DROP_ROT, FLAG_DROP_TRANS, FLAG_UB_INF = 1, 2, 4, 8

EXPORTS = ["gosma_create", "gosma_destroy", "gosma_last_error", "gosma_set_mixtures", "gosma_set_domain",
           "gosma_set_problems", "gosma_get_S22", "gosma_eval_bounds", "gosma_solve", "gosma_solve_batch",
           "gosma_set_timing", "gosma_get_timing", "gosma_get_trace", "gosma_mlp_init", "gosma_mlp_set_params",
           "gosma_mlp_get_params", "gosma_mlp_predict", "gosma_mlp_loss_grad", "gosma_mlp_train",
           "gosma_set_record_sink", "gosma_get_tiles", "gosma_set_tiles", "gosma_autotune", "gosma_get_work_counts",
           "gosma_snapshot", "gosma_resume", "gosma_refine", "gosma_dpmeans", "gosma_dpvmf_means",
           "gosma_eval_bounds_noalloc", "gosma_get_bucket_tiles", "gosma_set_kappa_pieces",
           "gosma_get_kappa_pieces"]
MLP_FEATURES, MLP_RECORD, MLP_PARAMS = 20, 21, 35841
NOALLOC_MAX_CUBES = 65536
N_BUCKETS = 4
KERNEL_KINDS = ["s11", "s12", "select", "branch", "push", "mlp", "sma"]
WORK_COUNTS = ["cubes", "s12_screened", "s12_evaluated", "cells", "s11_screened", "s11_evaluated"]


class GosmaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Domain(C.Structure):
    _fields_ = [("r_lo", C.c_double * 3), ("r_hi", C.c_double * 3), ("t_lo", C.c_double * 3),
                ("t_hi", C.c_double * 3), ("zeta", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("batch_parents", C.c_int64), ("max_queue", C.c_int64),
                ("max_iters", C.c_int64), ("time_limit_s", C.c_double), ("order", C.c_int),
                ("log_records", C.c_int), ("trace_every", C.c_int), ("no_graph", C.c_int),
                ("learned_window", C.c_double), ("sma_iters", C.c_int)]


class Tile(C.Structure):
    _fields_ = [("waves", C.c_int32), ("blocks", C.c_int32)]


class Tiles(C.Structure):
    _fields_ = [("s11", Tile), ("s12", Tile)]


class Result(C.Structure):
    _fields_ = [("f_best", C.c_double), ("lb_global", C.c_double), ("f_norm_best", C.c_double),
                ("lb_norm", C.c_double), ("r", C.c_double * 3), ("t", C.c_double * 3), ("iters", C.c_int64),
                ("cubes", C.c_int64), ("max_queue_used", C.c_int64), ("seconds", C.c_double),
                ("status", C.c_int), ("sma_runs", C.c_int64), ("sma_improved", C.c_int64)]


_lib = None


def lib():
    """Load libgosma.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1812_01232_amd.build")
        L = C.CDLL(str(LIB_PATH))
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
        L.gosma_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.gosma_destroy.argtypes = [vp]
        L.gosma_destroy.restype = None
        L.gosma_last_error.argtypes = [vp]
        L.gosma_last_error.restype = C.c_char_p
        L.gosma_set_mixtures.argtypes = [vp, C.c_int, dp, dp, dp, ip, C.c_int, dp, dp, dp, ip, C.c_int]
        L.gosma_set_domain.argtypes = [vp, C.POINTER(Domain)]
        L.gosma_set_problems.argtypes = [vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64), dp, dp, dp, ip,
                                         dp, dp, dp, ip, C.c_int, C.POINTER(Domain)]
        L.gosma_get_S22.argtypes = [vp, C.c_int, dp]
        L.gosma_eval_bounds.argtypes = [vp, vp, vp, vp, C.c_int64, vp, vp, vp, vp, vp, vp]
        L.gosma_eval_bounds_noalloc.argtypes = [vp, vp, vp, vp, C.c_int64, vp, vp, vp, vp, vp, vp]
        L.gosma_solve.argtypes = [vp, C.POINTER(Opts), C.POINTER(Result)]
        L.gosma_solve_batch.argtypes = [vp, C.POINTER(Opts), C.POINTER(Result)]
        L.gosma_set_timing.argtypes = [vp, C.c_int]
        L.gosma_get_trace.argtypes = [vp, dp, C.c_int64, C.POINTER(C.c_int64)]
        fp = C.POINTER(C.c_float)
        L.gosma_mlp_init.argtypes = [vp, C.c_uint64]
        L.gosma_mlp_set_params.argtypes = [vp, fp]
        L.gosma_mlp_get_params.argtypes = [vp, fp]
        L.gosma_mlp_predict.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.gosma_mlp_loss_grad.argtypes = [vp, vp, C.c_int64, dp, fp]
        L.gosma_mlp_train.argtypes = [vp, vp, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_uint64, fp]
        L.gosma_set_record_sink.argtypes = [vp, vp, C.c_int64, vp]
        L.gosma_get_timing.argtypes = [vp, dp, C.POINTER(C.c_int64)]
        L.gosma_get_work_counts.argtypes = [vp, C.POINTER(C.c_int64)]
        L.gosma_snapshot.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.gosma_resume.argtypes = [vp, vp, C.c_size_t]
        L.gosma_get_tiles.argtypes = [vp, C.POINTER(Tiles)]
        L.gosma_get_bucket_tiles.argtypes = [vp, C.c_int, C.POINTER(Tiles), C.POINTER(C.c_int)]
        L.gosma_set_tiles.argtypes = [vp, C.POINTER(Tiles)]
        L.gosma_set_kappa_pieces.argtypes = [vp, C.c_int]
        L.gosma_get_kappa_pieces.argtypes = [vp]
        L.gosma_autotune.argtypes = [vp, C.c_int64, C.c_uint64, dp, C.c_int64, C.POINTER(C.c_int64),
                                     C.POINTER(Tiles)]
        L.gosma_refine.argtypes = [vp, C.c_int64, C.POINTER(C.c_uint32), dp, dp, C.c_int, dp, dp, dp, dp, ip]
        for name in ("gosma_dpmeans", "gosma_dpvmf_means"):
            getattr(L, name).argtypes = [vp, vp, C.c_int64, C.c_double, C.c_int, C.c_int, C.c_double, vp, dp,
                                         C.POINTER(C.c_int64), dp, C.POINTER(C.c_int), C.POINTER(C.c_int), vp]
        _lib = L
    return _lib


def _d(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def domain_of(scene):
    return Domain((C.c_double * 3)(*scene.r_lo), (C.c_double * 3)(*scene.r_hi), (C.c_double * 3)(*scene.t_lo),
                  (C.c_double * 3)(*scene.t_hi), float(scene.zeta))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One libgosma context bound to a HIP device."""

    def __init__(self, device=0):
        self._h = C.c_void_p()
        self._check(lib().gosma_create(int(device), C.byref(self._h)), "gosma_create")
        self.device = device

    def close(self):
        if self._h:
            lib().gosma_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc, what):
        if rc != GOSMA_OK:
            msg = lib().gosma_last_error(self._h).decode() if self._h else what
            raise GosmaError(rc, f"{what}: {msg}")

    # -- problems ---------------------------------------------------------
    def set_scene(self, scene):
        """Set the single problem from a scene (mixtures + domain)."""
        self._keep = [_f64(scene.mu), _f64(scene.sigma), _f64(scene.phi1), _i32(scene.label1),
                      _f64(scene.dir2), _f64(scene.kappa2), _f64(scene.phi2), _i32(scene.label2)]
        mu, sg, p1, l1, d2, k2, p2, l2 = self._keep
        self._check(lib().gosma_set_mixtures(self._h, mu.shape[0], _d(mu), _d(sg), _d(p1), _i(l1), d2.shape[0],
                                             _d(d2), _d(k2), _d(p2), _i(l2), int(scene.n_labels)),
                    "gosma_set_mixtures")
        dom = domain_of(scene)
        self._check(lib().gosma_set_domain(self._h, C.byref(dom)), "gosma_set_domain")

    def set_scenes(self, scenes_list):
        """Set several independent problems (the batched form)."""
        go = np.cumsum([0] + [s.M for s in scenes_list]).astype(np.int64)
        vo = np.cumsum([0] + [s.N for s in scenes_list]).astype(np.int64)
        cat = lambda f: _f64(np.concatenate([getattr(s, f) for s in scenes_list]))
        labelled = scenes_list[0].label1 is not None
        if any((s.label1 is not None) != labelled or s.n_labels != scenes_list[0].n_labels for s in scenes_list):
            raise ValueError("the problems of one batch must all be labelled with the same number of classes, "
                             "or all unlabelled")
        l1 = _i32(np.concatenate([s.label1 for s in scenes_list])) if labelled else None
        l2 = _i32(np.concatenate([s.label2 for s in scenes_list])) if labelled else None
        doms = (Domain * len(scenes_list))(*[domain_of(s) for s in scenes_list])
        self._keep = [go, vo, cat("mu"), cat("sigma"), cat("phi1"), l1, cat("dir2"), cat("kappa2"), cat("phi2"),
                      l2, doms]
        _, _, mu, sg, p1, _, d2, k2, p2, _, _ = self._keep
        self._check(lib().gosma_set_problems(self._h, len(scenes_list), go.ctypes.data_as(C.POINTER(C.c_int64)),
                                             vo.ctypes.data_as(C.POINTER(C.c_int64)), _d(mu), _d(sg), _d(p1),
                                             _i(l1), _d(d2), _d(k2), _d(p2), _i(l2),
                                             int(scenes_list[0].n_labels), doms), "gosma_set_problems")

    def S22(self, problem=0):
        v = C.c_double()
        self._check(lib().gosma_get_S22(self._h, int(problem), C.byref(v)), "gosma_get_S22")
        return v.value

    # -- bounds -----------------------------------------------------------
    def eval_bounds(self, rkeys, tkeys, ub, lb, flags, aux=None, top8=None, problem=None, stream=None):
        """Tensors in/out (see gosma_eval_bounds: device memory is used in place, host
        memory is staged by the library); runs on the current stream."""
        n = int(rkeys.numel())
        s = _current_stream() if stream is None else C.c_void_p(stream)
        self._check(lib().gosma_eval_bounds(self._h, _ptr(rkeys), _ptr(tkeys), _ptr(problem), n, _ptr(ub), _ptr(lb),
                                            _ptr(flags), _ptr(aux), _ptr(top8), s), "gosma_eval_bounds")

    def eval_bounds_noalloc(self, rkeys, tkeys, ub, lb, flags, aux=None, top8=None, problem=None, stream=None):
        """gosma_eval_bounds_noalloc: device tensors only, at most NOALLOC_MAX_CUBES
        cubes; the library allocates nothing; runs on the current stream."""
        n = int(rkeys.numel())
        s = _current_stream() if stream is None else C.c_void_p(stream)
        self._check(lib().gosma_eval_bounds_noalloc(self._h, _ptr(rkeys), _ptr(tkeys), _ptr(problem), n, _ptr(ub),
                                                    _ptr(lb), _ptr(flags), _ptr(aux), _ptr(top8), s),
                    "gosma_eval_bounds_noalloc")

    def bounds(self, rkeys_np, tkeys_np, problem_np=None, want_aux=True, want_top8=False):
        """Convenience: host keys in, host arrays out (copies through torch)."""
        import torch
        dev = torch.device("cuda", self.device)
        n = len(rkeys_np)
        rk = torch.from_numpy(np.ascontiguousarray(rkeys_np, dtype=np.uint64).view(np.int64)).to(dev)
        tk = torch.from_numpy(np.ascontiguousarray(tkeys_np, dtype=np.uint64).view(np.int64)).to(dev)
        pr = None
        if problem_np is not None:
            pr = torch.from_numpy(np.ascontiguousarray(problem_np, dtype=np.uint32).view(np.int32)).to(dev)
        ub = torch.empty(n, dtype=torch.float64, device=dev)
        lb = torch.empty(n, dtype=torch.float64, device=dev)
        fl = torch.empty(n, dtype=torch.uint8, device=dev)
        aux = torch.empty(n, 4, dtype=torch.float64, device=dev) if want_aux else None
        t8 = torch.empty(n, 8, dtype=torch.float32, device=dev) if want_top8 else None
        self.eval_bounds(rk, tk, ub, lb, fl, aux, t8, pr)
        torch.cuda.synchronize(dev)
        out = {"ub": ub.cpu().numpy(), "lb": lb.cpu().numpy(), "flags": fl.cpu().numpy()}
        if want_aux:
            out["aux"] = aux.cpu().numpy()
        if want_top8:
            out["top8"] = t8.cpu().numpy()
        return out

    def bounds_host(self, rkeys_np, tkeys_np, problem_np=None, want_aux=True, want_top8=False):
        """Host (numpy) arrays straight through the C-ABI: the library copies
        them to and from the device itself; synchronous."""
        n = len(rkeys_np)
        rk = np.ascontiguousarray(rkeys_np, dtype=np.uint64)
        tk = np.ascontiguousarray(tkeys_np, dtype=np.uint64)
        pr = None if problem_np is None else np.ascontiguousarray(problem_np, dtype=np.uint32)
        out = {"ub": np.empty(n), "lb": np.empty(n), "flags": np.empty(n, np.uint8)}
        if want_aux:
            out["aux"] = np.empty((n, 4))
        if want_top8:
            out["top8"] = np.empty((n, 8), np.float32)
        p = lambda a: None if a is None else C.c_void_p(a.ctypes.data)
        self._check(lib().gosma_eval_bounds(self._h, p(rk), p(tk), p(pr), n, p(out["ub"]), p(out["lb"]),
                                            p(out["flags"]), p(out.get("aux")), p(out.get("top8")), None),
                    "gosma_eval_bounds")
        return out

    # -- local refinement (SMA) ---------------------------------------------
    def refine(self, r0, t0, max_iters=100, problem=None, want_grad=True):
        """SMA from each start (rows of r0, t0): {"r", "t", "f", "grad", "iters"};
        max_iters = 0 evaluates the objective and its gradient at the starts."""
        r0 = _f64(np.atleast_2d(r0))
        t0 = _f64(np.atleast_2d(t0))
        n = r0.shape[0]
        r, t, f = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n)
        g = np.zeros((n, 6)) if want_grad else None
        it = np.zeros(n, dtype=np.int32)
        pr = None
        if problem is not None:
            pr = np.ascontiguousarray(problem, dtype=np.uint32)
        self._check(lib().gosma_refine(self._h, n, None if pr is None else pr.ctypes.data_as(C.POINTER(C.c_uint32)),
                                       _d(r0), _d(t0), int(max_iters), _d(r), _d(t), _d(f), _d(g), _i(it)),
                    "gosma_refine")
        return {"r": r, "t": t, "f": f, "grad": g, "iters": it}

    # -- mixture generation (clustering + ML fits) ----------------------------
    def _cluster(self, fn, name, x, lam, max_clusters, max_passes, clamp):
        import torch
        dev = torch.device("cuda", self.device)
        xt = x if isinstance(x, torch.Tensor) else torch.from_numpy(_f64(x))
        xt = xt.to(dev, dtype=torch.float64).contiguous()
        n = int(xt.shape[0])
        lab = torch.empty(n, dtype=torch.int32, device=dev)
        mu = np.zeros((max_clusters, 3))
        cnt = np.zeros(max_clusters, dtype=np.int64)
        sp = np.zeros(max_clusters)
        K, passes = C.c_int(), C.c_int()
        torch.cuda.synchronize(dev)
        self._check(fn(self._h, _ptr(xt), n, float(lam), int(max_clusters), int(max_passes), float(clamp), _ptr(lab),
                       _d(mu), cnt.ctypes.data_as(C.POINTER(C.c_int64)), _d(sp), C.byref(K), C.byref(passes),
                       _current_stream()), name)
        k = K.value
        return {"K": k, "labels": lab.cpu().numpy(), "centres": mu[:k].copy(), "counts": cnt[:k].copy(),
                "spread": sp[:k].copy(), "passes": passes.value}

    def dpmeans(self, points, lam, max_clusters=1024, max_passes=100, sigma_min=1e-3):
        """DP-means + isotropic Gaussian fit: {K, labels, centres, counts, spread (sigma), passes}."""
        return self._cluster(lib().gosma_dpmeans, "gosma_dpmeans", points, lam, max_clusters, max_passes, sigma_min)

    def dpvmf_means(self, dirs, cos_lam, max_clusters=1024, max_passes=100, kappa_max=1e5):
        """DP-vMF-means + vMF fit: {K, labels, centres, counts, spread (kappa), passes}."""
        return self._cluster(lib().gosma_dpvmf_means, "gosma_dpvmf_means", dirs, cos_lam, max_clusters, max_passes,
                             kappa_max)

    # -- queue-ordering network -------------------------------------------
    def mlp_init(self, seed=0):
        self._check(lib().gosma_mlp_init(self._h, int(seed)), "gosma_mlp_init")

    def mlp_set_params(self, theta):
        p = np.ascontiguousarray(theta, dtype=np.float32)
        assert p.size == MLP_PARAMS
        self._check(lib().gosma_mlp_set_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float))), "gosma_mlp_set_params")

    def mlp_get_params(self):
        p = np.zeros(MLP_PARAMS, dtype=np.float32)
        self._check(lib().gosma_mlp_get_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float))), "gosma_mlp_get_params")
        return p

    def _dev(self, a):
        import torch
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.device("cuda", self.device))

    def mlp_predict(self, X):
        import torch
        x = self._dev(X)
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        self._check(lib().gosma_mlp_predict(self._h, _ptr(x), x.shape[0], _ptr(y), _current_stream()),
                    "gosma_mlp_predict")
        torch.cuda.synchronize(x.device)
        return y.cpu().numpy().astype(np.float64)

    def mlp_loss_grad(self, X, t):
        import torch
        rec = self._dev(np.concatenate([np.asarray(X), np.asarray(t)[:, None]], axis=1))
        torch.cuda.synchronize(rec.device)
        loss = C.c_double()
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        self._check(lib().gosma_mlp_loss_grad(self._h, _ptr(rec), rec.shape[0], C.byref(loss),
                                              g.ctypes.data_as(C.POINTER(C.c_float))), "gosma_mlp_loss_grad")
        return loss.value, g.astype(np.float64)

    def mlp_train(self, X=None, t=None, records=None, epochs=10, batch=4096, lr=1e-3, seed=0):
        """Train on records (device tensor n x 21) or on host arrays X, t."""
        import torch
        if records is None:
            records = self._dev(np.concatenate([np.asarray(X), np.asarray(t)[:, None]], axis=1))
        torch.cuda.synchronize(records.device)
        hist = np.zeros(max(int(epochs), 1), dtype=np.float32)
        self._check(lib().gosma_mlp_train(self._h, _ptr(records), int(records.shape[0]), int(epochs), int(batch),
                                          float(lr), int(seed), hist.ctypes.data_as(C.POINTER(C.c_float))),
                    "gosma_mlp_train")
        return hist.astype(np.float64)

    def set_record_sink(self, records, count):
        """records: device float32 tensor [capacity, 21]; count: device int64 tensor [1] (zeroed)."""
        cap = 0 if records is None else int(records.shape[0])
        self._check(lib().gosma_set_record_sink(self._h, _ptr(records), cap, _ptr(count)), "gosma_set_record_sink")

    # -- reading of the kappa dependence of the lower bound -----------------
    def set_kappa_pieces(self, m):
        """Pieces of the kappa interval in the S12 upper term (1, 2 or 4; see gosma.h)."""
        self._check(lib().gosma_set_kappa_pieces(self._h, int(m)), "gosma_set_kappa_pieces")

    def get_kappa_pieces(self):
        return int(lib().gosma_get_kappa_pieces(self._h))

    # -- launch shapes of the bound kernels ---------------------------------
    def get_tiles(self):
        """{"s11": (waves, blocks), "s12": (waves, blocks)}"""
        t = Tiles()
        self._check(lib().gosma_get_tiles(self._h, C.byref(t)), "gosma_get_tiles")
        return {"s11": (t.s11.waves, t.s11.blocks), "s12": (t.s12.waves, t.s12.blocks)}

    def set_tiles(self, s11, s12):
        t = Tiles(Tile(*s11), Tile(*s12))
        self._check(lib().gosma_set_tiles(self._h, C.byref(t)), "gosma_set_tiles")

    def autotune(self, n_cubes=32768, seed=0):
        """Time the candidate launch shapes on random cubes and keep the fastest, for
        all problems and per size bucket.  Returns {"chosen": get_tiles(), "buckets":
        {bucket: bucket_tiles(bucket)} for the non-empty buckets, "table": [(kernel,
        waves, blocks, ms, bucket), ...]} (bucket -1: all problems)."""
        cap = 30 * (1 + N_BUCKETS)
        rows = np.zeros((cap, 5))
        n = C.c_int64()
        t = Tiles()
        self._check(lib().gosma_autotune(self._h, int(n_cubes), int(seed), _d(rows), cap, C.byref(n),
                                         C.byref(t)), "gosma_autotune")
        table = [(KERNEL_KINDS[int(r[0])], int(r[1]), int(r[2]), float(r[3]), int(r[4])) for r in rows[:min(n.value, cap)]]
        buckets = {}
        for k in range(N_BUCKETS):
            bt = self.bucket_tiles(k)
            if bt["n_problems"]:
                buckets[k] = bt
        return {"chosen": {"s11": (t.s11.waves, t.s11.blocks), "s12": (t.s12.waves, t.s12.blocks)}, "buckets": buckets,
                "table": table}

    def bucket_tiles(self, bucket):
        """{"s11": (waves, blocks), "s12": (...), "n_problems": n} of a size bucket."""
        t = Tiles()
        n = C.c_int()
        self._check(lib().gosma_get_bucket_tiles(self._h, int(bucket), C.byref(t), C.byref(n)), "gosma_get_bucket_tiles")
        return {"s11": (t.s11.waves, t.s11.blocks), "s12": (t.s12.waves, t.s12.blocks), "n_problems": n.value}

    # -- kernel timing ----------------------------------------------------
    def set_timing(self, enable=True):
        self._check(lib().gosma_set_timing(self._h, int(bool(enable))), "gosma_set_timing")

    def get_timing(self):
        """{kind: (total ms, launches)} since the last call; synchronises."""
        ms = (C.c_double * 8)()
        n = (C.c_int64 * 8)()
        self._check(lib().gosma_get_timing(self._h, ms, n), "gosma_get_timing")
        return {KERNEL_KINDS[k]: (ms[k], n[k]) for k in range(len(KERNEL_KINDS))}

    def get_work_counts(self):
        """Work counts of the timed launches since the last call (live cubes,
        GMM-vMF pairs screened and evaluated, translation cells, GMM-GMM
        pairs screened and evaluated); synchronises."""
        c = (C.c_int64 * len(WORK_COUNTS))()
        self._check(lib().gosma_get_work_counts(self._h, c), "gosma_get_work_counts")
        return {k: int(c[i]) for i, k in enumerate(WORK_COUNTS)}

    def get_pair_counts(self):
        """(screened, evaluated) GMM-vMF pairs of the timed launches since the
        last call; synchronises (and clears every work count)."""
        w = self.get_work_counts()
        return w["s12_screened"], w["s12_evaluated"]

    # -- branch and bound -------------------------------------------------
    def solve(self, eps, batch_parents=4096, max_queue=1 << 24, max_iters=0, time_limit_s=0.0, order=0,
              log_records=0, trace_every=0, no_graph=False, learned_window=0.0, allow_overflow=False, sma_iters=0):
        """With allow_overflow a full queue returns the result (status 3) instead of raising."""
        o = Opts(eps, batch_parents, max_queue, max_iters, time_limit_s, order, log_records, trace_every,
                 int(bool(no_graph)), float(learned_window), int(sma_iters))
        r = Result()
        rc = lib().gosma_solve(self._h, C.byref(o), C.byref(r))
        if not (allow_overflow and rc == QUEUE_OVERFLOW):
            self._check(rc, "gosma_solve")
        return _result_dict(r)

    def trace(self):
        """Rows {iteration, seconds, cubes, queue, d*, min lb} of the last traced solve."""
        n = C.c_int64()
        self._check(lib().gosma_get_trace(self._h, None, 0, C.byref(n)), "gosma_get_trace")
        buf = np.zeros((max(n.value, 1), 6))
        self._check(lib().gosma_get_trace(self._h, _d(buf), n.value, C.byref(n)), "gosma_get_trace")
        return buf[:n.value]

    def solve_batch(self, n_problems, eps, batch_parents=2048, max_queue=1 << 22, max_iters=0, time_limit_s=0.0,
                    order=0, no_graph=False, learned_window=0.0, allow_overflow=False, sma_iters=0):
        """With allow_overflow problems whose queue filled up come back with status 3 instead of raising."""
        o = Opts(eps, batch_parents, max_queue, max_iters, time_limit_s, order, 0, 0, int(bool(no_graph)),
                 float(learned_window), int(sma_iters))
        rs = (Result * n_problems)()
        rc = lib().gosma_solve_batch(self._h, C.byref(o), rs)
        if not (allow_overflow and rc == QUEUE_OVERFLOW):
            self._check(rc, "gosma_solve_batch")
        return [_result_dict(r) for r in rs]

    # -- checkpoint of the search -------------------------------------------
    def snapshot(self):
        """The search state left by the last solve, as bytes."""
        n = C.c_size_t(0)
        self._check(lib().gosma_snapshot(self._h, None, C.byref(n)), "gosma_snapshot")
        buf = (C.c_uint8 * n.value)()
        self._check(lib().gosma_snapshot(self._h, buf, C.byref(n)), "gosma_snapshot")
        return bytes(buf[:n.value])

    def resume(self, data):
        """The next solve starts from this snapshot (None discards a pending one)."""
        if data is None:
            self._check(lib().gosma_resume(self._h, None, 0), "gosma_resume")
            return
        b = bytes(data)
        self._check(lib().gosma_resume(self._h, C.c_char_p(b), len(b)), "gosma_resume")


def _result_dict(r):
    return {name: (list(getattr(r, name)) if name in ("r", "t") else getattr(r, name)) for name, _ in Result._fields_}
