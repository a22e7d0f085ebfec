"""gosma_eval_bounds_noalloc against gosma_eval_bounds, through the C-ABI.

The allocation-free entry point runs the same kernels with their per-cube
scratch in the library's fixed device array, so on the same cubes and launch
shape its outputs must equal the allocating entry point's bit for bit (the
bar for this pair is stricter than the oracle tolerance).  Two calls in a
row, the second smaller, so that the second reads scratch the first left
behind; then the 16 x 16 results are also held to the FP64 oracle, and the
entry point's errors are checked (size limit, host arrays).
"""
import ctypes

import numpy as np
import pytest

import oracle
from synth import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_01232_amd import Context
    c = Context(0)
    yield c
    c.close()


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a).view(dtype)).to("cuda:0")


def _run(ctx, rk, tk, pr, noalloc, top8=True):
    n = len(rk)
    d = torch.device("cuda", 0)
    out = dict(ub=torch.full((n,), -7.0, dtype=torch.float64, device=d),
               lb=torch.full((n,), -7.0, dtype=torch.float64, device=d),
               flags=torch.full((n,), 0xEE, dtype=torch.uint8, device=d),
               aux=torch.full((n, 4), -7.0, dtype=torch.float64, device=d),
               top8=torch.full((n, 8), -7.0, dtype=torch.float32, device=d) if top8 else None)
    rkd, tkd = _dev(rk, np.int64), _dev(tk, np.int64)
    prd = None if pr is None else _dev(pr.astype(np.uint32), np.int32)
    f = ctx.eval_bounds_noalloc if noalloc else ctx.eval_bounds
    f(rkd, tkd, out["ub"], out["lb"], out["flags"], out["aux"], out["top8"], prd)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def _same(a, b, label):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), f"{label}: {k} differs"


def test_noalloc_matches_allocating_entry_point_two_calls(ctx):
    sc = scenes.cfg1_scene(0)
    ctx.set_scene(sc)
    rk, tk = scenes.random_cubes(sc, 6000, 1700)
    print(f"no-alloc: 16x16 scene, calls of 6000 then 1500 cubes", flush=True)
    first_na = _run(ctx, rk, tk, None, True)
    first = _run(ctx, rk, tk, None, False)
    _same(first_na, first, "first call")
    # the second call is smaller and reads scratch the first one wrote
    rk2, tk2 = rk[3000:4500], tk[3000:4500]
    second_na = _run(ctx, rk2, tk2, None, True, top8=False)
    second = _run(ctx, rk2, tk2, None, False, top8=False)
    _same(second_na, second, "second call")
    # and both agree with the oracle to the parity tolerance
    o = oracle.OracleProblem(sc).bounds(rk2, tk2)
    ok = o["status"] == 0
    assert np.array_equal(ok, (second_na["flags"] & 6) == 0)
    fin = ok & np.isfinite(o["ub"])
    sc_ub = o["s11_ub"] + 2 * o["s12_ub"]
    sc_lb = o["s11_lo"] + 2 * o["s12_hi"]
    assert np.all(np.abs(second_na["ub"][fin] - o["ub"][fin]) <= TOL * sc_ub[fin])
    assert np.all(np.abs(second_na["lb"][ok] - o["lb"][ok]) <= TOL * sc_lb[ok])


def test_noalloc_batched_problems_at_capacity(ctx):
    # several problems (vMF rows staged in LDS), at the array's full capacity
    from paper_1812_01232_amd.gosma import NOALLOC_MAX_CUBES
    scs = scenes.batch_scenes(6, seed=4100)
    ctx.set_scenes(scs)
    n = NOALLOC_MAX_CUBES
    rks, tks, prs = [], [], []
    per = n // len(scs)
    for p, s in enumerate(scs):
        rk, tk = scenes.random_cubes(s, per + (n - per * len(scs) if p == 0 else 0), 1800 + p)
        rks.append(rk)
        tks.append(tk)
        prs.append(np.full(len(rk), p, np.uint32))
    rk, tk, pr = np.concatenate(rks), np.concatenate(tks), np.concatenate(prs)
    assert len(rk) == n
    print(f"no-alloc: 6 problems, {n} cubes, then {n // 3}", flush=True)
    a = _run(ctx, rk, tk, pr, True, top8=False)
    b = _run(ctx, rk, tk, pr, False, top8=False)
    _same(a, b, "full capacity")
    sl = slice(n // 3, 2 * n // 3)
    a = _run(ctx, rk[sl], tk[sl], pr[sl], True, top8=False)
    b = _run(ctx, rk[sl], tk[sl], pr[sl], False, top8=False)
    _same(a, b, "smaller second call")


def test_noalloc_rejects_oversize_and_host_arrays(ctx):
    from paper_1812_01232_amd import gosma
    sc = scenes.cfg1_scene(0)
    ctx.set_scene(sc)
    n = gosma.NOALLOC_MAX_CUBES + 1
    d = torch.device("cuda", 0)
    rk = torch.zeros(n, dtype=torch.int64, device=d)
    ub = torch.empty(n, dtype=torch.float64, device=d)
    lb = torch.empty(n, dtype=torch.float64, device=d)
    fl = torch.empty(n, dtype=torch.uint8, device=d)
    L = gosma.lib()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = L.gosma_eval_bounds_noalloc(ctx._h, p(rk), p(rk), None, n, p(ub), p(lb), p(fl), None, None, None)
    assert rc == -1 and b"GOSMA_NOALLOC_MAX_CUBES" in L.gosma_last_error(ctx._h)
    # host arrays are not staged (staging would allocate): rejected
    h = np.zeros(4, np.uint64)
    hu = np.zeros(4)
    hp = lambda a: ctypes.c_void_p(a.ctypes.data)
    rc = L.gosma_eval_bounds_noalloc(ctx._h, hp(h), hp(h), None, 4, hp(hu), hp(hu), hp(h), None, None, None)
    assert rc == -1 and b"device memory" in L.gosma_last_error(ctx._h)


@pytest.mark.parametrize("m", [2, 4])
def test_noalloc_with_kappa_pieces(ctx, m):
    # the kappa-pieces reading goes through the allocation-free entry point too
    sc = scenes.cfg2_scene(0)
    ctx.set_scene(sc)
    rk, tk = scenes.random_cubes(sc, 3000, 1900 + m)
    print(f"no-alloc: 64x64 scene, kappa pieces {m}, 3000 then 1000 cubes", flush=True)
    try:
        ctx.set_kappa_pieces(m)
        a = _run(ctx, rk, tk, None, True, top8=False)
        b = _run(ctx, rk, tk, None, False, top8=False)
        _same(a, b, f"kappa pieces {m}")
        a = _run(ctx, rk[500:1500], tk[500:1500], None, True, top8=False)
        b = _run(ctx, rk[500:1500], tk[500:1500], None, False, top8=False)
        _same(a, b, f"kappa pieces {m}, smaller second call")
        # the top-8 output is defined for the one-piece term only
        with pytest.raises(RuntimeError, match="kappa pieces"):
            _run(ctx, rk[:64], tk[:64], None, True, top8=True)
    finally:
        ctx.set_kappa_pieces(1)
    # the pieces change the lower bound only: flags as with one piece, upper
    # bounds to FP32 rounding (the two kernels may fuse multiply-adds apart)
    one = _run(ctx, rk[500:1500], tk[500:1500], None, True, top8=False)
    assert np.array_equal(a["flags"], one["flags"])
    fin = np.isfinite(one["ub"])
    assert np.array_equal(np.isfinite(a["ub"]), fin)
    assert np.all(np.abs(a["ub"][fin] - one["ub"][fin]) <= 1e-6 * np.abs(one["ub"][fin]))
