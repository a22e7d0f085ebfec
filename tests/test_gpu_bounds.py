"""Parity of the HIP bound evaluation with the FP64 oracle.

Element-wise on the same seeded cubes: drop flags exactly, the upper and
lower bounds to 1e-5 of their own scale (S11 + 2 S12 of that bound: a
relative tolerance on S11 - 2 S12 itself is ill-conditioned where the two
sums nearly cancel), the branching flag wherever the two uncertainty angles
it compares differ by more than rounding, and the top-8 pair terms.
"""
import math

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


def _compare(sc, g, o, top8=False, label=""):
    drop_o = o["status"] != 0
    drop_g = (g["flags"] & 6) != 0
    assert np.array_equal(drop_o, drop_g), f"{label}: drop flags differ"
    assert np.array_equal(o["status"] == 1, (g["flags"] & 2) != 0)
    ok = ~drop_o
    assert np.all(np.isinf(g["ub"][drop_o])) and np.all(np.isinf(g["lb"][drop_o]))
    inf_o = ok & ~np.isfinite(o["ub"])
    assert np.array_equal(inf_o, ok & ((g["flags"] & 8) != 0)), f"{label}: infeasible-centre flags differ"
    fin = ok & ~inf_o
    sc_ub = o["s11_ub"] + 2 * o["s12_ub"]
    sc_lb = o["s11_lo"] + 2 * o["s12_hi"]
    e_ub = np.abs(g["ub"][fin] - o["ub"][fin]) / sc_ub[fin]
    e_lb = np.abs(g["lb"][ok] - o["lb"][ok]) / sc_lb[ok]
    worst_ub = e_ub.max(initial=0.0)
    worst_lb = e_lb.max(initial=0.0)
    print(f"{label}: n={len(ok)} ok={ok.sum()} worst ub err {worst_ub:.2e} lb err {worst_lb:.2e}")
    assert worst_ub <= TOL, f"{label}: ub error {worst_ub}"
    assert worst_lb <= TOL, f"{label}: lb error {worst_lb}"
    # components of the sums
    aux = g["aux"]
    assert np.all(np.abs(aux[fin, 0] - o["s11_ub"][fin]) <= TOL * sc_ub[fin])
    assert np.all(np.abs(aux[fin, 1] - o["s12_ub"][fin]) <= TOL * sc_ub[fin])
    assert np.all(np.abs(aux[ok, 2] - o["s11_lo"][ok]) <= TOL * sc_lb[ok])
    assert np.all(np.abs(aux[ok, 3] - o["s12_hi"][ok]) <= TOL * sc_lb[ok])
    # branching flag where it is decided by more than rounding
    gap = o["psi_r"] - o["psi_t_mean"]
    clear = ok & (np.abs(gap) > 1e-5)
    assert np.array_equal((g["flags"][clear] & 1) != 0, o["split_rot"][clear] != 0)
    if top8:
        t = g["top8"][fin].astype(np.float64)
        assert np.all(np.abs(t - o["top8"][fin]) <= TOL * sc_ub[fin, None])
    return ok


def test_cfg1_bound_pass_65536(ctx):
    """The cfg1 bound pass: 65,536 random sub-cubes, every one checked."""
    sc = scenes.cfg1_scene(0)
    rk, tk = scenes.random_cubes(sc, 65536, 1500)
    ctx.set_scene(sc)
    g = ctx.bounds(rk, tk, want_top8=True)
    o = oracle.OracleProblem(sc).bounds(rk, tk)
    ok = _compare(sc, g, o, top8=True, label="cfg1")
    assert ok.sum() > 50000


@pytest.mark.parametrize("idx", [0, 1])
def test_cfg2_random_cubes(ctx, idx):
    sc = scenes.cfg2_scene(idx)
    rk, tk = scenes.random_cubes(sc, 3000, 2500 + idx)
    ctx.set_scene(sc)
    g = ctx.bounds(rk, tk, want_top8=True)
    o = oracle.OracleProblem(sc).bounds(rk, tk)
    _compare(sc, g, o, top8=True, label=f"cfg2-{idx}")


def test_cfg2_full_batch_sampled(ctx):
    """The 32,768-cube cfg2 batch in one launch; a seeded sample of 1,500
    cubes is checked against the oracle one by one."""
    sc = scenes.cfg2_scene(0)
    rk, tk = scenes.random_cubes(sc, 32768, 2600, r_levels=(2, 12), t_levels=(1, 10))
    ctx.set_scene(sc)
    g = ctx.bounds(rk, tk)
    sel = np.random.default_rng(0).choice(32768, 1500, replace=False)
    o = oracle.OracleProblem(sc).bounds(rk[sel], tk[sel])
    gs = {k: v[sel] for k, v in g.items()}
    _compare(sc, gs, o, label="cfg2-full")


def test_cfg3_labels_sampled(ctx):
    sc = scenes.cfg3_scene(0)
    rk, tk = scenes.random_cubes(sc, 4096, 3500, r_levels=(2, 12), t_levels=(1, 10))
    ctx.set_scene(sc)
    g = ctx.bounds(rk, tk, want_top8=True)
    sel = np.random.default_rng(1).choice(4096, 300, replace=False)
    o = oracle.OracleProblem(sc).bounds(rk[sel], tk[sel])
    _compare(sc, {k: v[sel] for k, v in g.items()}, o, top8=True, label="cfg3")


def test_cfg3_full_launch_sampled(ctx):
    """The 256 x 256 labelled workload at its full batch: 131,072 cubes in one
    launch of each kernel (every block walks 16 cubes at 8,192 blocks), with
    400 cubes spread over the batch, its last cubes included, checked
    against the oracle."""
    sc = scenes.cfg3_scene(0)
    n = 131072
    rk, tk = scenes.random_cubes(sc, n, 3600, r_levels=(2, 12), t_levels=(1, 10))
    ctx.set_scene(sc)
    for tile in [(1, 8192), (2, 8192)]:
        ctx.set_tiles(s11=tile, s12=tile)
        g = ctx.bounds(rk, tk, want_top8=True)
        sel = np.concatenate([np.random.default_rng(3).choice(n - 16, 384, replace=False), np.arange(n - 16, n)])
        o = oracle.OracleProblem(sc).bounds(rk[sel], tk[sel])
        _compare(sc, {k: v[sel] for k, v in g.items()}, o, top8=True, label=f"cfg3-full tile {tile}")


def test_cfg4_128_problems_sampled(ctx):
    """The 128-problem batch (M, N uniform on [16, 256]) at its search size:
    16,384 cubes per problem (256 seeded cubes, each repeated 64 times), 2.1 M
    cubes in one launch of each kernel, under the benchmark's launch shape and
    one-wave blocks; four cubes per problem are checked against the oracle."""
    scs = scenes.batch_scenes(128, seed=4000)
    ctx.set_scenes(scs)
    uniq, per = 256, 16384
    rks, tks, want = [], [], []
    for p, s in enumerate(scs):
        rk, tk = scenes.random_cubes(s, uniq, 6000 + p, r_levels=(2, 12), t_levels=(1, 10))
        rks.append(np.tile(rk, per // uniq))
        tks.append(np.tile(tk, per // uniq))
        want.append(oracle.OracleProblem(s).bounds(rk[:4], tk[:4]))
    rk, tk = np.concatenate(rks), np.concatenate(tks)
    pid = np.repeat(np.arange(128, dtype=np.uint32), per)
    for tile in [(4, 8192), (1, 8192)]:
        ctx.set_tiles(s11=tile, s12=tile)
        g = ctx.bounds(rk, tk, problem_np=pid)
        for p, s in enumerate(scs):
            # the sampled cubes and their last copies in the launch
            for off in (0, per - uniq):
                m = np.arange(p * per + off, p * per + off + 4)
                _compare(s, {k: v[m] for k, v in g.items()}, want[p], label=f"cfg4-{p} tile {tile} copy {off}")


def test_cubes_around_true_pose(ctx):
    """Deep cubes containing the true pose (the cubes that decide termination)."""
    sc = scenes.cfg2_scene(0)
    keys = []
    for Lr in range(2, 19, 2):
        for Lt in range(1, 18, 2):
            ir = np.clip(np.floor((sc.r_gt - sc.r_lo) / (sc.r_hi - sc.r_lo) * 2 ** Lr), 0, 2 ** Lr - 1).astype(int)
            it = np.clip(np.floor((sc.t_gt - sc.t_lo) / (sc.t_hi - sc.t_lo) * 2 ** Lt), 0, 2 ** Lt - 1).astype(int)
            keys.append((int(scenes.pack_key(Lr, *ir)), int(scenes.pack_key(Lt, *it))))
    rk = np.array([k[0] for k in keys], np.uint64)
    tk = np.array([k[1] for k in keys], np.uint64)
    ctx.set_scene(sc)
    g = ctx.bounds(rk, tk)
    o = oracle.OracleProblem(sc).bounds(rk, tk)
    _compare(sc, g, o, label="around-gt")


def test_edge_cases(ctx):
    # root cube, level-19 cubes, dropped rotation cells, infeasible translations,
    # single components, odd class sizes
    sc = scenes.small_scene(1, 1, seed=3)
    rk = np.array([0, int(scenes.pack_key(19, 262144, 300000, 1)), int(scenes.pack_key(3, 7, 7, 7)),
                   int(scenes.pack_key(1, 1, 0, 1))], np.uint64)
    tk = np.array([0, int(scenes.pack_key(19, 5, 524287, 77)), 0, int(scenes.pack_key(2, 3, 0, 1))], np.uint64)
    ctx.set_scene(sc)
    g = ctx.bounds(rk, tk)
    o = oracle.OracleProblem(sc).bounds(rk, tk)
    _compare(sc, g, o, label="edge-1x1")
    sc2 = scenes.small_scene(7, 5, seed=4, n_labels=3, n_inliers=4)
    sc2.mu[0] = np.array([0.01, 0.02, -0.03])
    rk2, tk2 = scenes.random_cubes(sc2, 2000, 4600, r_levels=(0, 19), t_levels=(0, 19))
    ctx.set_scene(sc2)
    g = ctx.bounds(rk2, tk2, want_top8=True)
    o = oracle.OracleProblem(sc2).bounds(rk2, tk2)
    _compare(sc2, g, o, top8=True, label="edge-labels")
    # the moved mean makes translation cells around it infeasible (every
    # vertex within zeta): both sides drop them
    assert (o["status"] == 2).sum() >= 100
    assert np.array_equal((g["flags"] & 4) != 0, o["status"] == 2)


def test_empty_batch_and_errors(ctx):
    from paper_1812_01232_amd import GosmaError
    sc = scenes.cfg1_scene(0)
    ctx.set_scene(sc)
    z = torch.empty(0, dtype=torch.int64, device="cuda")
    d = torch.empty(0, dtype=torch.float64, device="cuda")
    f = torch.empty(0, dtype=torch.uint8, device="cuda")
    ctx.eval_bounds(z, z, d, d, f)       # n = 0 is a no-op
    bad = scenes.cfg1_scene(0)
    bad.sigma = bad.sigma.copy()
    bad.sigma[3] = -1.0
    with pytest.raises(GosmaError):
        ctx.set_scene(bad)


@pytest.mark.parametrize("tile,labelled", [(None, False), (None, True), ((1, 3), False), ((2, 2048), True),
                                           ((4, 1024), False)])
def test_batched_problems(ctx, tile, labelled):
    """Several problems of different sizes in one launch, problem index per
    cube; with several problems the pair kernel stages each cube's vMF rows in
    LDS, on every launch shape.  Labelled batches: three classes each."""
    if labelled:
        scs = [scenes.small_scene(m, n, seed=4107 + m, noise_deg=1.0, n_inliers=3 * min(m, n) // 4,
                                  sigma=(0.05, 0.3), t_half=1.0, room=((-5, -5, -1.5), (5, 5, 1.5)), n_labels=3)
               for m, n in [(40, 50), (24, 17), (64, 64), (33, 70), (16, 16), (90, 45)]]
        with pytest.raises(ValueError):   # one class count for the whole batch
            ctx.set_scenes(scenes.batch_scenes(2, seed=4100, lo=16, hi=32) + scs[:1])
    else:
        scs = scenes.batch_scenes(6, seed=4100, lo=16, hi=96)
    ctx.set_scenes(scs)
    if tile is not None:
        ctx.set_tiles(s11=tile, s12=tile)
    rks, tks, pids = [], [], []
    for p, s in enumerate(scs):
        rk, tk = scenes.random_cubes(s, 300, 4700 + p, r_levels=(1, 10), t_levels=(0, 9))
        rks.append(rk)
        tks.append(tk)
        pids.append(np.full(300, p, np.uint32))
    perm = np.random.default_rng(2).permutation(1800)
    rk = np.concatenate(rks)[perm]
    tk = np.concatenate(tks)[perm]
    pid = np.concatenate(pids)[perm]
    g = ctx.bounds(rk, tk, problem_np=pid)
    for p, s in enumerate(scs):
        m = pid == p
        o = oracle.OracleProblem(s).bounds(rk[m], tk[m])
        _compare(s, {k: v[m] for k, v in g.items()}, o, label=f"batch-{p} tile {tile}")
        assert ctx.S22(p) == pytest.approx(oracle.OracleProblem(s).S22(), rel=1e-12)


def test_deterministic(ctx):
    sc = scenes.cfg2_scene(1)
    rk, tk = scenes.random_cubes(sc, 4096, 2700)
    ctx.set_scene(sc)
    a = ctx.bounds(rk, tk)
    b = ctx.bounds(rk, tk)
    assert np.array_equal(a["ub"], b["ub"]) and np.array_equal(a["lb"], b["lb"])


TILES = [(1, 8192), (2, 2048), (4, 1024), (4, 7), (2, 5), (1, 3)]


@pytest.mark.parametrize("M,N", [(64, 64), (40, 32), (70, 128), (33, 45), (100, 256)])
def test_launch_shapes_and_pair_mappings(ctx, M, N):
    """Every launch shape (waves per block, grid size) on vMF counts that hit
    each pair mapping: a multiple of the block (broadcast rows), a divisor of
    it, and neither (flattened rectangle); all against the oracle, and the
    shapes against each other to FP64 summation order."""
    sc = scenes.small_scene(M, N, seed=M * 1000 + N, noise_deg=1.0, n_inliers=min(N, 3 * M // 4),
                            sigma=(0.05, 0.3), t_half=1.0, room=((-5, -5, -1.5), (5, 5, 1.5)))
    rk, tk = scenes.random_cubes(sc, 600, 5100 + M + N, r_levels=(1, 14), t_levels=(0, 12))
    ctx.set_scene(sc)
    o = oracle.OracleProblem(sc).bounds(rk, tk)
    first = None
    for t in TILES:
        ctx.set_tiles(s11=t, s12=t)
        assert ctx.get_tiles() == {"s11": t, "s12": t}
        g = ctx.bounds(rk, tk, want_top8=True)
        _compare(sc, g, o, top8=True, label=f"{M}x{N} tile {t}")
        if first is None:
            first = g
        else:
            fin = np.isfinite(first["ub"])
            scale = np.abs(first["aux"][:, 0]) + 2 * np.abs(first["aux"][:, 1])
            assert np.all(np.abs(g["ub"][fin] - first["ub"][fin]) <= 1e-6 * scale[fin])
            assert np.array_equal(g["flags"], first["flags"])


def test_autotune(ctx):
    """The autotuner times 3 x 5 shapes per kernel, keeps one of them, and the
    bounds under the chosen shapes still match the oracle."""
    sc = scenes.cfg2_scene(0)
    ctx.set_scene(sc)
    res = ctx.autotune(n_cubes=8192, seed=1)
    table = res["table"]
    # all problems (bucket -1), then the one size bucket of the 64x64 problem
    assert len(table) == 60 and sorted({r[4] for r in table}) == [-1, 0]
    for kind in ("s11", "s12"):
        for bk in (-1, 0):
            rows = [r for r in table if r[0] == kind and r[4] == bk]
            assert len(rows) == 15 and all(r[3] > 0 for r in rows)
            best = min(rows, key=lambda r: r[3])
            got = res["chosen"][kind] if bk < 0 else res["buckets"][0][kind]
            assert got == (best[1], best[2])
    assert ctx.get_tiles() == res["chosen"]
    assert list(res["buckets"]) == [0]
    print("autotune chosen", res["chosen"])
    rk, tk = scenes.random_cubes(sc, 1000, 2800, r_levels=(2, 12), t_levels=(1, 10))
    g = ctx.bounds(rk, tk)
    _compare(sc, g, oracle.OracleProblem(sc).bounds(rk, tk), label="after-autotune")
    from paper_1812_01232_amd import GosmaError
    with pytest.raises(GosmaError):
        ctx.set_tiles(s11=(3, 10), s12=(1, 10))
    with pytest.raises(GosmaError):
        ctx.set_tiles(s11=(1, 0), s12=(1, 10))


@pytest.mark.parametrize("M,N", [(1024, 1024), (2500, 700), (4096, 4096)])
def test_max_components(ctx, M, N):
    """Large mixtures up to the largest the library accepts, M = N = 4096.
    Up to about 1,600 components the bound kernels stage each cube's records
    in LDS (96 bytes per GMM component); beyond, in the context's global
    record buffer.  A few cubes checked one by one, and SMA's objective and
    gradient at two poses."""
    sc = scenes.small_scene(M, N, seed=77, noise_deg=1.0, n_inliers=int(0.7 * min(M, N)), sigma=(0.05, 0.3),
                            t_half=1.0, room=((-5, -5, -1.5), (5, 5, 1.5)))
    n = 12 if M <= 1024 else 6
    rk, tk = scenes.random_cubes(sc, n, 5300, r_levels=(2, 12), t_levels=(1, 10))
    ctx.set_scene(sc)
    P = oracle.OracleProblem(sc)
    o = P.bounds(rk, tk)
    for t in [(1, 64), (4, 64)]:
        ctx.set_tiles(s11=t, s12=t)
        g = ctx.bounds(rk, tk)
        _compare(sc, g, o, label=f"{M}x{N} tile {t}")
    r0 = np.stack([sc.r_gt, sc.r_gt + 0.1])
    t0 = np.stack([sc.t_gt, np.clip(sc.t_gt + 0.1, sc.t_lo, sc.t_hi)])
    out = ctx.refine(r0, t0, max_iters=0)
    for s in range(2):
        if out["iters"][s] < 0:
            continue
        fo, go = P.objective_grad(r0[s], t0[s])
        _, s11, s12 = P.objective(r0[s], t0[s])
        assert abs(out["f"][s] - fo) <= 1e-5 * (s11 + 2 * s12)
        assert np.max(np.abs(out["grad"][s] - go)) <= 1e-4 * np.max(np.abs(go)) + 1e-5 * (s11 + 2 * s12)


def test_pair_screen_counts_and_parity(ctx):
    """The screen of negligible GMM-vMF pairs: every same-class pair of a live
    cube is screened, most of them are dropped on deep cubes (where the
    uncertainty angles are small), none on the root cube, and the bounds of
    the same cubes still match the oracle (dropped pairs are counted at the
    threshold, 1e-9 of the bound scale in all)."""
    sc = scenes.cfg2_scene(0)
    ctx.set_scene(sc)
    for levels, lo_frac, hi_frac in [((10, 12), 0.0, 0.6), ((0, 0), 1.0, 1.0)]:
        rk, tk = scenes.random_cubes(sc, 2000, 5900, r_levels=levels, t_levels=(levels[0] - 1 if levels[0] else 0,
                                                                              levels[1] - 1 if levels[1] else 0))
        ctx.get_work_counts()
        ctx.set_timing(True)
        g = ctx.bounds(rk, tk)
        ctx.set_timing(False)
        ctx.get_timing()
        w = ctx.get_work_counts()
        screened, evaluated = w["s12_screened"], w["s12_evaluated"]
        live = int(((g["flags"] & 6) == 0).sum())
        assert w["cubes"] == live
        assert screened == live * sc.M * sc.N
        # every cube's translation cell is its own cell here; those not dropped
        # for zeta are counted with all their unordered GMM pairs
        assert w["s11_screened"] == w["cells"] * sc.M * (sc.M - 1) // 2
        assert w["cells"] >= live and w["s11_evaluated"] <= w["s11_screened"]
        frac = evaluated / screened
        print(f"levels {levels}: {live} live cubes, {frac:.3f} of the pairs evaluated")
        assert lo_frac <= frac <= hi_frac
        o = oracle.OracleProblem(sc).bounds(rk, tk)
        _compare(sc, g, o, label=f"screen {levels}")


def test_host_arrays_through_the_abi(ctx):
    """Host arrays handed to gosma_eval_bounds are staged by the library and
    give the device path's results bit for bit; pinned host memory and mixed
    host/device arguments too; a larger call after a smaller one grows the
    staging buffers."""
    sc = scenes.cfg1_scene(0)
    ctx.set_scene(sc)
    for n, seed in [(1000, 1601), (5000, 1602)]:
        rk, tk = scenes.random_cubes(sc, n, seed)
        dev = ctx.bounds(rk, tk, want_top8=True)
        host = ctx.bounds_host(rk, tk, want_top8=True)
        for key in ("ub", "lb", "flags", "aux", "top8"):
            assert np.array_equal(dev[key], host[key], equal_nan=True), (n, key)
    # pinned host inputs, device outputs
    n = 777
    rk, tk = scenes.random_cubes(sc, n, 1603)
    ref = ctx.bounds(rk, tk)
    prk = torch.from_numpy(rk.view(np.int64)).pin_memory()
    ptk = torch.from_numpy(tk.view(np.int64)).pin_memory()
    ub = torch.empty(n, dtype=torch.float64, device="cuda")
    lb = torch.empty(n, dtype=torch.float64, device="cuda")
    fl = torch.empty(n, dtype=torch.uint8, device="cuda")
    ctx.eval_bounds(prk, ptk, ub, lb, fl)
    torch.cuda.synchronize()
    assert np.array_equal(ub.cpu().numpy(), ref["ub"]) and np.array_equal(lb.cpu().numpy(), ref["lb"])
    assert np.array_equal(fl.cpu().numpy(), ref["flags"])


@pytest.mark.parametrize("m", [2, 4])
def test_kappa_pieces_match_oracle(ctx, m):
    """The tighter reading of the kappa dependence (the S12 upper term's kappa
    interval in m pieces) against the oracle's same reading, on one problem
    and on a batch of problems (vMF rows staged in LDS); the upper bounds do
    not change, and the lower bounds are at least the one-piece ones on most
    cubes."""
    sc = scenes.cfg2_scene(0)
    rk, tk = scenes.random_cubes(sc, 800, 7700 + m, r_levels=(2, 12), t_levels=(1, 10))
    ctx.set_scene(sc)
    P = oracle.OracleProblem(sc)
    g1 = ctx.bounds(rk, tk)
    try:
        ctx.set_kappa_pieces(m)
        oracle.set_kappa_pieces(m)
        assert ctx.get_kappa_pieces() == m
        g = ctx.bounds(rk, tk)
        o = P.bounds(rk, tk)
        _compare(sc, g, o, label=f"cfg2 kappa pieces {m}")
        # the same upper-bound formula in both kernels; their FP32 pair terms
        # may round apart where the compiler fuses multiply-adds differently
        fin = np.isfinite(g1["ub"])
        assert np.array_equal(np.isfinite(g["ub"]), fin)
        assert np.all(np.abs(g["ub"][fin] - g1["ub"][fin]) <= 1e-6 * np.abs(g1["ub"][fin]))
        ok = (g1["flags"] & 6) == 0
        assert np.mean(g["lb"][ok] >= g1["lb"][ok] - 1e-6 * np.abs(g1["lb"][ok])) >= 0.8
        with pytest.raises(RuntimeError, match="kappa pieces"):
            ctx.bounds(rk[:8], tk[:8], want_top8=True)   # the pieces need no top-8 terms
        scs = scenes.batch_scenes(3, seed=4300 + m, lo=16, hi=80)
        ctx.set_scenes(scs)
        ctx.set_kappa_pieces(m)
        for p, s in enumerate(scs):
            rkp, tkp = scenes.random_cubes(s, 64, 7800 + p, r_levels=(2, 10), t_levels=(1, 8))
            gp = ctx.bounds(np.concatenate([rkp, rkp]), np.concatenate([tkp, tkp]),
                            problem_np=np.full(128, p, np.uint32))
            op = oracle.OracleProblem(s).bounds(rkp, tkp)
            _compare(s, {k: v[:64] for k, v in gp.items()}, op, label=f"batch {p} kappa pieces {m}")
    finally:
        ctx.set_kappa_pieces(1)
        oracle.set_kappa_pieces(1)
    with pytest.raises(RuntimeError, match="kappa pieces"):
        ctx.set_kappa_pieces(3)
