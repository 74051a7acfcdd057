"""GPU path (libwos through its C ABI) against the CPU oracle.

Both sides draw the same Philox4x32-10 streams, so walks are the same up to
rounding.  In FP64 the walks agree step for step: exit counts must match
exactly and the matrices to summation-order rounding.  In FP32 a walk can
take a different branch where its FP32 position decides a comparison
differently (the eps test, a near-tie between two centres); the comparison
there is statistical, against the oracle's own Monte Carlo standard errors.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle.volume import cell_counts
from oracle.walker import build_toolbox as oracle_build, site_events, bin_site

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2608_07017_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu_tb(dom, sites, bnodes, walks, eps, seed, **kw):
    _say("GPU build:", dom["kind"], "n=%d p=%d N=%d eps=%g" % (len(sites), len(bnodes), walks, eps), kw)
    tb = P.Toolbox(dom, sites, bnodes, walks, eps, seed=seed, **kw)
    tb.build()
    torch.cuda.synchronize()
    return tb


def _np(t):
    return t.detach().cpu().numpy()


def _export_all(tb):
    out = {k: _np(tb.export(k)) for k in ("A", "B", "H", "K", "Hcount", "lambda", "vcount")}
    out["Hcount"] = out["Hcount"].astype(np.int64)
    return out


# ---------------------------------------------------------------- volume


@pytest.mark.parametrize("name,dom", [("disk", W.unit_disk()), ("lshape", W.l_shape()),
                                      ("ball", W.unit_ball()), ("cubeball", W.cube_minus_ball())])
def test_volume_counts_bit_exact(name, dom):
    sites = W.sample_sites(dom, 57, 3, 1e-3)
    bn = sites[:5]    # any centres: only the volume stream is checked here
    npts = (1 << 19) + 3   # ragged: the last Philox block is partly used
    tb = _gpu_tb(dom, sites, bn, 1, 1e-3, 777, precision="f64", volume_samples=npts)
    got = _np(tb.export("vcount")).astype(np.int64)
    ref = cell_counts(dom, sites, 777, npts)
    assert np.array_equal(got, ref)
    lam = _np(tb.export("lambda"))
    assert np.allclose(lam, ref / ref.sum(), rtol=1e-15, atol=0)
    assert tb.info()["volume_inside"] == ref.sum()


# ---------------------------------------------------------- FP64 walker


def _compare_f64(dom, sites, bn, walks, eps, seed, **kw):
    tb = _gpu_tb(dom, sites, bn, walks, eps, seed, precision="f64", volume_samples=1 << 12, **kw)
    g = _export_all(tb)
    info = tb.info()
    ref = oracle_build(dom, sites, bn, walks, eps, seed, fixed_M=kw.get("fixed_M", 0),
                       max_steps=kw.get("max_steps", 0) or 10000)
    assert info["walks"] == len(sites) * walks
    assert info["walk_steps"] == ref["walk_steps"].sum()
    # per site: every walk takes the same number of steps as the oracle's
    assert np.array_equal(_np(tb.export("site_steps")), ref["walk_steps"])
    assert info["max_walk_steps"] == ref["max_steps"].max()
    assert info["capped_walks"] == ref["capped"].sum()
    assert np.array_equal(g["Hcount"], ref["Hcount"])
    for key in ("A", "B", "K"):
        scale = np.abs(ref[key]).max()
        assert np.allclose(g[key], ref[key], rtol=1e-10, atol=1e-12 * scale), key
    assert np.allclose(g["H"], ref["H"], rtol=1e-15, atol=0)
    return tb, g, ref


def test_disk64_fp64_full_size():
    """The 2-D unit-disk configuration at its full size: 64 sites, 64 boundary
    nodes, 2000 walks per site, eps 1e-3, FP64."""
    c = W.config("disk64")
    _compare_f64(c["domain"], c["sites"], c["bnodes"], c["walks"], c["eps"], c["seed"])


def test_ragged_multi_item_and_regeneration_schedules():
    """37 sites, 333 walks split in items of 100 (atomic flush path, ragged last
    item); the result must not depend on the lane schedule."""
    dom = W.unit_disk()
    sites = W.sample_sites(dom, 37, 5, 1e-3)
    bn = W.circle_nodes(19)
    tb1, g1, _ = _compare_f64(dom, sites, bn, 333, 1e-3, 42, walks_per_item=100, regen_threshold=1)
    tb2 = _gpu_tb(dom, sites, bn, 333, 1e-3, 42, precision="f64", volume_samples=1 << 12,
                  walks_per_item=333, regen_threshold=64)
    g2 = _export_all(tb2)
    assert np.array_equal(g1["Hcount"], g2["Hcount"])
    for key in ("A", "B", "K"):
        assert np.allclose(g1[key], g2[key], rtol=1e-12, atol=1e-15)


def test_single_walk_and_single_site():
    dom = W.unit_disk()
    _compare_f64(dom, np.array([[0.2, -0.3]]), W.circle_nodes(7), 1, 1e-3, 9)


def test_paper_fixed_M_mode():
    sites, bn = W.paper_square_layout()
    _compare_f64(W.unit_square(), sites[::13], bn, 200, 0.0, 3, fixed_M=30)


def test_per_estimator_walks_and_steps():
    """Per-estimator (M, N): A and B from 200 walks of 30 steps (seed 3),
    H and K from 500 walks of 60 steps (seed 8), combined by copying the
    second toolbox's H and K into the first; each must match the oracle
    build with its own (M, N, seed)."""
    sites, bn = W.paper_square_layout()
    s = sites[::13]
    dom = W.unit_square()
    tb1 = _gpu_tb(dom, s, bn, 200, 0.0, 3, precision="f64", volume_samples=1 << 12, fixed_M=30)
    tb2 = _gpu_tb(dom, s, bn, 500, 0.0, 8, precision="f64", volume_samples=1 << 12, fixed_M=60)
    tb1.take(tb2, "HK")
    g = _export_all(tb1)
    ref_ab = oracle_build(dom, s, bn, 200, 0.0, 3, fixed_M=30)
    ref_hk = oracle_build(dom, s, bn, 500, 0.0, 8, fixed_M=60)
    for key, ref in (("A", ref_ab), ("B", ref_ab), ("K", ref_hk)):
        scale = np.abs(ref[key]).max()
        assert np.allclose(g[key], ref[key], rtol=1e-10, atol=1e-12 * scale), key
    assert np.array_equal(g["Hcount"], ref_hk["Hcount"])
    assert np.allclose(g["H"], ref_hk["H"], rtol=1e-15, atol=0)
    # the source toolbox is unchanged, and a toolbox on other sites is refused
    assert np.array_equal(_export_all(tb2)["Hcount"], ref_hk["Hcount"])
    tb3 = _gpu_tb(dom, sites[1::13], bn, 10, 0.0, 3, precision="f64", volume_samples=1 << 12, fixed_M=5)
    with pytest.raises(P.WosError):
        tb1.take(tb3, "A")


@pytest.mark.parametrize("m", [25, 61])
def test_separate_v_partition_fp64(m):
    """W != V: 40 W centres (the walks' starts), m V centres (coarser and
    finer), FP64.  The matrices against the oracle's build on the same V
    centres, exit counts exactly; lambda over W and |V_j| / |D| over V both
    bit-exact against the oracle's binning of the same volume stream."""
    dom = W.unit_disk()
    sites = W.sample_sites(dom, 40, 31, 1e-3)
    vc = W.sample_sites(dom, m, 32, 1e-3)
    bn = W.circle_nodes(30)
    npts = 1 << 14
    _say("GPU build W != V: n=40 m=%d" % m)
    tb = P.Toolbox(dom, sites, bn, 300, 1e-3, seed=13, precision="f64", volume_samples=npts, vcentres=vc)
    tb.build()
    torch.cuda.synchronize()
    g = _export_all(tb)
    assert g["A"].shape == (40, m) and g["B"].shape == (2, 40, m)
    ref = oracle_build(dom, sites, bn, 300, 1e-3, 13, vcentres=vc)
    assert np.array_equal(g["Hcount"], ref["Hcount"])
    for key in ("A", "B", "K"):
        scale = np.abs(ref[key]).max()
        assert np.allclose(g[key], ref[key], rtol=1e-10, atol=1e-12 * scale), key
    cw = cell_counts(dom, sites, 13, npts)
    cv = cell_counts(dom, vc, 13, npts)
    assert np.array_equal(g["vcount"].astype(np.int64), cw)
    assert np.allclose(g["lambda"], cw / cw.sum(), rtol=1e-15, atol=0)
    assert np.allclose(_np(tb.export("lambda_v")), cv / cv.sum(), rtol=1e-15, atol=0)
    # routes not supported with n != m are refused
    with pytest.raises(P.WosError):
        tb.solve(np.ones(40), np.zeros(30), kind="semilinear_cubic")
    with pytest.raises(P.WosError):
        tb.operator()


def test_lambert_sampler_fp64():
    """The exact d = 2 radial sampler (Lambert W): A, B against the oracle's
    build with the same sampler (scipy's W_{-1} there, Halley's iteration on
    the GPU); the walks do not depend on the sampler, so the exit counts
    equal the default build's.  Refused in 3-D."""
    dom = W.unit_disk()
    sites = W.sample_sites(dom, 37, 5, 1e-3)
    bn = W.circle_nodes(19)
    tb, g, _ = _compare_f64_sampler(dom, sites, bn)
    with pytest.raises(P.WosError):
        P.Toolbox(W.unit_ball(), W.sample_sites(W.unit_ball(), 3, 1, 1e-3), W.fibonacci_sphere(8), 10, 1e-3,
                  precision="f64", sampler="lambert")


def _compare_f64_sampler(dom, sites, bn):
    tb = _gpu_tb(dom, sites, bn, 333, 1e-3, 42, precision="f64", volume_samples=1 << 12, sampler="lambert")
    g = _export_all(tb)
    ref = oracle_build(dom, sites, bn, 333, 1e-3, 42, sampler="lambert")
    base = oracle_build(dom, sites, bn, 333, 1e-3, 42)
    assert np.array_equal(g["Hcount"], ref["Hcount"]) and np.array_equal(ref["Hcount"], base["Hcount"])
    for key in ("A", "B", "K"):
        scale = np.abs(ref[key]).max()
        assert np.allclose(g[key], ref[key], rtol=1e-10, atol=1e-12 * scale), key
    # the estimators change (another sampler), their row sums agree in mean
    assert not np.allclose(g["A"], base["A"])
    return tb, g, ref


def test_step_cap_counts():
    dom = W.unit_disk()
    sites = W.sample_sites(dom, 9, 8, 1e-2)
    _compare_f64(dom, sites, W.circle_nodes(12), 300, 1e-9, 4, max_steps=6)


@pytest.mark.parametrize("name", ["ball3d", "lshape", "cubeball"])
def test_other_domains_fp64(name):
    if name == "ball3d":
        dom, bn = W.unit_ball(), W.fibonacci_sphere(48)
    elif name == "lshape":
        dom = W.l_shape()
        bn = W.polygon_nodes(dom["verts"], 40)
    else:
        dom = W.cube_minus_ball()
        bn = np.concatenate([W.cube_face_nodes(4), W.fibonacci_sphere(30, dom["center"], dom["radius"])])
    sites = W.sample_sites(dom, 23, 11, 1e-3)
    _compare_f64(dom, sites, bn, 400, 1e-4, 17)


# ------------------------------------------------ tallies straight to HBM


@pytest.mark.parametrize("case", ["disk", "ragged", "cubeball"])
def test_hbm_tally_mode_fp64(case):
    """The walker mode that adds every tally into the toolbox in device memory
    (used when a site's rows do not fit in LDS), forced on small cases: the
    same walks, so exit counts exact and the matrices to rounding."""
    if case == "disk":
        c = W.config("disk64")
        _compare_f64(c["domain"], c["sites"][:40], c["bnodes"], 500, c["eps"], c["seed"], tally="hbm")
    elif case == "ragged":
        dom = W.unit_disk()
        sites = W.sample_sites(dom, 37, 5, 1e-3)
        _compare_f64(dom, sites, W.circle_nodes(19), 333, 1e-3, 42, walks_per_item=100, tally="hbm")
    else:
        dom = W.cube_minus_ball()
        bn = np.concatenate([W.cube_face_nodes(4), W.fibonacci_sphere(30, dom["center"], dom["radius"])])
        sites = W.sample_sites(dom, 23, 11, 1e-3)
        _compare_f64(dom, sites, bn, 300, 1e-4, 17, tally="hbm")


def test_hbm_tally_fp32_matches_lds_tally():
    """FP32 walker: the two tally modes run the same walks; exit counts equal,
    the matrices equal to FP32 summation rounding."""
    dom = W.unit_square()
    sites = W.sample_sites(dom, 96, 21, 1e-3)
    bn = W.square_nodes(16)
    g1 = _export_all(_gpu_tb(dom, sites, bn, 3000, 1e-4, 5, precision="f32", volume_samples=1 << 14))
    g2 = _export_all(_gpu_tb(dom, sites, bn, 3000, 1e-4, 5, precision="f32", volume_samples=1 << 14,
                             tally="hbm"))
    assert np.array_equal(g1["Hcount"], g2["Hcount"])
    for key in ("A", "B", "K"):
        mass = np.abs(g1[key]).sum(axis=-1, keepdims=True)
        assert np.all(np.abs(g1[key] - g2[key]) <= 1e-5 * mass), key


@pytest.mark.parametrize("case", ["square", "lshape", "ball", "cubeball"])
def test_window_tally_fp32_matches_lds_rows(case):
    """The windowed tally mode (V cells and boundary cells ranked along a
    Morton curve, a few pages per site in LDS, the rest by device atomics,
    columns put back in the caller's order) forced with small windows, so
    that both paths carry many tallies, against the LDS-row mode on the same
    walks: exit counts equal, the matrices equal to FP32 summation rounding,
    the walk statistics identical."""
    dom = {"square": W.unit_square(), "lshape": W.l_shape(), "ball": W.unit_ball(),
           "cubeball": W.cube_minus_ball()}[case]
    d = dom["dim"]
    sites = W.sample_sites(dom, 333, 23, 1e-3)          # 6 pages, the last one ragged
    if case == "square":
        bn = W.square_nodes(40)
    elif case == "lshape":
        bn = W.polygon_nodes(dom["verts"], 150)
    elif case == "ball":
        bn = W.fibonacci_sphere(150)
    else:
        bn = np.concatenate([W.cube_face_nodes(4), W.fibonacci_sphere(54, dom["center"], dom["radius"])])
    kw = dict(precision="f32", volume_samples=1 << 12)
    t1 = _gpu_tb(dom, sites, bn, 2000, 1e-4, 13, **kw)
    t2 = _gpu_tb(dom, sites, bn, 2000, 1e-4, 13, tally="window", window_pages=2, window_bpages=1, **kw)
    i1, i2 = t1.info(), t2.info()
    for k in ("walks", "walk_steps", "max_walk_steps", "capped_walks"):
        assert i1[k] == i2[k], k
    g1, g2 = _export_all(t1), _export_all(t2)
    _same_walks_fp32(g1, g2, len(sites) * 2000)
    # a second build on the same toolbox (the accumulators start from zero again)
    t2.build(seed=13)
    torch.cuda.synchronize()
    g3 = _export_all(t2)
    assert np.array_equal(g3["Hcount"].sum(1), g2["Hcount"].sum(1))
    _same_walks_fp32(g3, g2, len(sites) * 2000)


def test_window_sites_split_by_their_own_bound():
    """In the windowed mode each site is split into items by its own
    fixed-point bound: a site 1e-6 from the boundary takes items of 526
    walks (8 items for 4000 walks), the others one item each, whose window
    is flushed with plain stores.  Against the LDS-row mode on the same
    walks."""
    dom = W.unit_square()
    sites = np.concatenate([W.sample_sites(dom, 40, 31, 1e-3), [[1e-6, 0.5]]])
    bn = W.square_nodes(24)
    # items of up to all 4000 walks: the 40 far sites take one item each
    wk = dict(tally="window", window_pages=1, window_bpages=1, walks_per_item=4000)
    plan = P.build_plan(dom, sites, bn, 4000, 1e-4, **wk)
    assert plan["items_per_site"] == 8 and plan["walks_per_item"] == int(0.49 * 2 ** 31 / 2e6)
    kw = dict(precision="f32", volume_samples=1 << 12)
    t1 = _gpu_tb(dom, sites, bn, 4000, 1e-4, 17, **kw)
    t2 = _gpu_tb(dom, sites, bn, 4000, 1e-4, 17, **wk, **kw)
    i1, i2 = t1.info(), t2.info()
    for k in ("walks", "walk_steps", "max_walk_steps", "capped_walks"):
        assert i1[k] == i2[k], k
    g1, g2 = _export_all(t1), _export_all(t2)
    # the row mode sums in FP64 here (the near site's bound is beyond fixed
    # point), the window in 2^-32 units: each tally is truncated by less than
    # 2^-32, so an entry may differ by up to the mean tallies per walk times
    # 2^-32 (the near site's A row, about 5e-13 in all, is below one unit)
    q = 2.0 ** -32 * (1 + i1["walk_steps"] / i1["walks"])
    _same_walks_fp32(g1, g2, len(sites) * 4000, atol=q)
    assert g2["A"][-1].max() <= q
    assert np.array_equal(g2["Hcount"].sum(1), np.full(len(sites), 4000))


def _same_walks_fp32(g1, g2, walks, atol=0.0):
    """Two FP32 toolboxes of the same walks whose binning visits tied
    centres in another order: every exit counted once in both, a walk binned
    to the other of two equidistant nodes at most about once per 1e5 walks
    (exact FP32 ties), and otherwise the matrices equal to summation
    rounding: the windowed sums are FP32 (relative rounding up to about
    1e-5 of a cell that takes thousands of tallies, such as a site's own),
    the row mode's exact fixed point."""
    h1, h2 = g1["Hcount"], g2["Hcount"]
    assert np.array_equal(h1.sum(1), h2.sum(1))
    moved = np.abs(h1 - h2).sum()
    assert moved <= 2 * max(4, 1e-5 * walks), moved
    tied = h1 != h2                                     # entries a tie moved an exit into or out of
    for key in ("A", "B"):
        mass = np.abs(g1[key]).sum(axis=-1, keepdims=True)
        assert np.all(np.abs(g1[key] - g2[key]) <= 1e-4 * mass + atol), key
    mass = np.abs(g1["K"]).sum(axis=-1, keepdims=True)
    ok = np.abs(g1["K"] - g2["K"]) <= 1e-4 * mass + atol
    assert np.all(ok | tied[None]), "K"
    # the row sums of K hold every exit's weight in both
    assert np.allclose(g1["K"].sum(-1), g2["K"].sum(-1), rtol=1e-4, atol=1e-4 * mass[..., 0].max())


def test_rows_beyond_lds_fp64_sampled():
    """7000 sites in FP64: a site's rows of A and B need 168 000 bytes, more
    than the 160 KiB of LDS, so the walker tallies into device memory.
    Sampled rows against the oracle's walks of those sites."""
    dom = W.unit_square()
    n = 7000
    sites = W.sample_sites(dom, n, 31, 1e-3)
    bn = W.square_nodes(16)
    walks, eps, seed = 40, 1e-3, 8
    tb = _gpu_tb(dom, sites, bn, walks, eps, seed, precision="f64", volume_samples=1 << 12)
    rows = np.array([0, 1, 2999, n // 2, n - 2, n - 1])
    A = _np(tb.export("A")[rows])
    B = _np(tb.export("B")[:, rows])
    K = _np(tb.export("K")[:, rows])
    Hc = _np(tb.export("Hcount")[rows]).astype(np.int64)
    steps = 0
    for r, i in enumerate(rows):
        ev = site_events(dom, sites[i], int(i), np.arange(walks), eps, seed)
        a, b, h, kk = bin_site(ev, sites, bn)
        steps += int(ev.nsteps.sum())
        assert np.array_equal(Hc[r], h.astype(np.int64))
        sc = np.abs(a).max() / walks
        assert np.allclose(A[r], a / walks, rtol=1e-10, atol=1e-12 * sc)
        for d in range(2):
            assert np.allclose(B[d, r], b[d] / walks, rtol=1e-10, atol=1e-12 * sc)
            assert np.allclose(K[d, r], kk[d] / walks, rtol=1e-10, atol=1e-12)
    assert tb.info()["walks"] == n * walks


# ---------------------------------------------------------- FP32 walker


def _row_functionals(A, B, H, K, g):
    ones = np.ones(A.shape[1])
    return {"A1": A @ ones, "B1": np.einsum("anm,m->an", B, ones), "Hg": H @ g,
            "Kg": np.einsum("anp,p->an", K, g)}


NBATCH = 32


def _oracle_rows_with_se(dom, sites, bn, walks, eps, seed, rows, g):
    """Oracle rows plus standard errors: per-walk SE of the four row
    functionals, and per entry SE_ij from NBATCH batch means (walk l in batch
    l mod NBATCH) of A, B, H and K, with the number of oracle tallies that
    fell in each entry."""
    from oracle.voronoi import nearest
    d = sites.shape[1]
    m, p = len(sites), len(bn)
    out = {k: [] for k in ("A", "B", "H", "K", "seA1", "seB1", "seHg", "seKg", "steps",
                           "seA", "seB", "seH", "seK", "hitA", "hitB", "hitH")}
    for i in rows:
        ev = site_events(dom, sites[i], int(i), np.arange(walks), eps, seed)
        a, b, h, kk = bin_site(ev, sites, bn)
        out["A"].append(a / walks)
        out["B"].append(b / walks)
        out["H"].append(h / walks)
        out["K"].append(kk / walks)
        N = walks
        cA = np.bincount(ev.ev_walk, weights=ev.ev_tA, minlength=N)
        cB = np.stack([np.bincount(ev.ev_walk, weights=ev.ev_tB[:, k], minlength=N) + ev.ball_w[:, k]
                       for k in range(d)], 1)
        jg = nearest(bn, ev.term_pts)
        gj = g[jg]
        out["seA1"].append(cA.std(ddof=1) / np.sqrt(N))
        out["seB1"].append(cB.std(axis=0, ddof=1) / np.sqrt(N))
        out["seHg"].append(gj.std(ddof=1) / np.sqrt(N))
        out["seKg"].append((ev.term_w * gj[:, None]).std(axis=0, ddof=1) / np.sqrt(N))
        out["steps"].append(ev.nsteps.sum())
        # batch means per entry
        bw = np.arange(N) % NBATCH
        nb = np.bincount(bw, minlength=NBATCH).astype(np.float64)
        jv = nearest(sites, ev.ev_pts)
        jb = nearest(sites, ev.ball_pts)
        be = ev.ev_walk % NBATCH
        sA = np.bincount(be * m + jv, weights=ev.ev_tA, minlength=NBATCH * m).reshape(NBATCH, m)
        sB = np.stack([np.bincount(be * m + jv, weights=ev.ev_tB[:, k], minlength=NBATCH * m).reshape(NBATCH, m)
                       + np.bincount(bw * m + jb, weights=ev.ball_w[:, k], minlength=NBATCH * m).reshape(NBATCH, m)
                       for k in range(d)])
        sH = np.bincount(bw * p + jg, minlength=NBATCH * p).reshape(NBATCH, p).astype(np.float64)
        sK = np.stack([np.bincount(bw * p + jg, weights=ev.term_w[:, k], minlength=NBATCH * p).reshape(NBATCH, p)
                       for k in range(d)])
        se = lambda sums: (sums / nb[:, None]).std(axis=-2, ddof=1) / np.sqrt(NBATCH)
        out["seA"].append(se(sA))
        out["seB"].append(np.stack([se(sB[k]) for k in range(d)]))
        out["seH"].append(se(sH))
        out["seK"].append(np.stack([se(sK[k]) for k in range(d)]))
        out["hitA"].append(np.bincount(jv, minlength=m))
        out["hitB"].append(np.bincount(jv, minlength=m) + np.bincount(jb, minlength=m))
        out["hitH"].append(np.bincount(jg, minlength=p))
    r = {k: np.array(v) for k, v in out.items()}
    for k in ("B", "K", "seB", "seK"):
        r[k] = r[k].transpose(1, 0, 2)
    return r


def _check_f32_rows(g, ref, rows, bn_g, site_steps=None):
    fg = _row_functionals(g["A"][rows], g["B"][:, rows], g["H"][rows], g["K"][:, rows], bn_g)
    fr = _row_functionals(ref["A"], ref["B"], ref["H"], ref["K"], bn_g)
    assert np.all(np.abs(fg["A1"] - fr["A1"]) <= 4 * ref["seA1"])
    assert np.all(np.abs(fg["B1"] - fr["B1"]) <= 4 * ref["seB1"].T)
    assert np.all(np.abs(fg["Hg"] - fr["Hg"]) <= 4 * ref["seHg"])
    assert np.all(np.abs(fg["Kg"] - fr["Kg"]) <= 4 * ref["seKg"].T)
    # entries, one by one: among the entries the oracle's
    # walks reached at least 10 times, at least 99.9 % within 4 SE_ij and all
    # within 6 SE_ij; the rest enter the moved-mass check below
    for key, hit in (("A", "hitA"), ("B", "hitB"), ("H", "hitH"), ("K", "hitH")):
        ga = g[key][rows] if key in ("A", "H") else g[key][:, rows]
        ra, se = ref[key], ref["se" + key]
        h = ref[hit] if key in ("A", "H") else np.broadcast_to(ref[hit], ra.shape)
        sel = h >= 10
        z = np.abs(ga - ra)[sel] / np.maximum(se[sel], 1e-300)
        assert np.mean(z <= 4) >= 0.999, (key, np.mean(z <= 4))
        assert np.all(z <= 6), (key, z.max())
        # the same walks up to FP32 branch flips, which move a few tallies
        # between neighbouring cells; the mass moved stays below 1 %
        moved = np.abs(ga - ra).sum(axis=-1)
        mass = np.abs(ra).sum(axis=-1)
        assert np.all(moved <= 0.01 * mass), (key, (moved / mass).max())
    # step counts: the walks take the oracle's steps up to rare FP32 flips of
    # the eps test (per-site totals agree to 1e-3)
    if site_steps is not None:
        rel = np.abs(site_steps - ref["steps"]) / ref["steps"]
        assert np.all(rel <= 1e-3), rel.max()


def test_square_fp32_small():
    dom = W.unit_square()
    sites = W.sample_sites(dom, 96, 21, 1e-3)
    bn = W.square_nodes(16)
    walks, eps, seed = 4000, 1e-4, 5
    tb = _gpu_tb(dom, sites, bn, walks, eps, seed, precision="f32", volume_samples=1 << 16)
    g = _export_all(tb)
    rows = np.arange(0, 96, 7)
    gb = bn[:, 0] ** 2 - bn[:, 1] ** 2
    ref = _oracle_rows_with_se(dom, sites, bn, walks, eps, seed, rows, gb)
    _check_f32_rows(g, ref, rows, gb, _np(tb.export("site_steps"))[rows])
    assert np.all(g["Hcount"].sum(axis=1) == walks)


def test_square1024_fp32_full_size_sampled_rows():
    """The 2-D unit-square configuration at full size, in the launch shape the
    benchmark times: 1024 sites, 256 boundary nodes, 1e4 walks, eps 1e-4, FP32.
    The oracle recomputes 6 sampled rows (rows are independent streams)."""
    c = W.config("square1024")
    tb = _gpu_tb(c["domain"], c["sites"], c["bnodes"], c["walks"], c["eps"], c["seed"], precision="f32")
    g = _export_all(tb)
    info = tb.info()
    assert info["walks"] == 1024 * 10000
    assert np.all(g["Hcount"].sum(axis=1) == c["walks"])          # each walk exits once
    rows = np.array([0, 1, 257, 511, 800, 1023])
    gb = c["bnodes"][:, 0] ** 2 - c["bnodes"][:, 1] ** 2
    ref = _oracle_rows_with_se(c["domain"], c["sites"], c["bnodes"], c["walks"], c["eps"], c["seed"], rows, gb)
    _check_f32_rows(g, ref, rows, gb, _np(tb.export("site_steps"))[rows])
    # harmonic extension of x^2 - y^2 at every site (accuracy, not parity):
    # bias from binning g on the boundary cells is O(h^2)
    hg = g["H"] @ gb
    exact = c["sites"][:, 0] ** 2 - c["sites"][:, 1] ** 2
    assert np.sqrt(np.mean((hg - exact) ** 2)) < 0.01


def _export_rows(tb, rows):
    """The sampled rows of every toolbox array, without copying whole
    matrices to the host (the 3-D configurations hold gigabytes)."""
    r = torch.as_tensor(rows, device="cuda")
    out = {k: _np(tb.export(k).index_select(0, r)) for k in ("A", "H", "Hcount")}
    out.update({k: _np(tb.export(k).index_select(1, r)) for k in ("B", "K")})
    out["Hcount"] = out["Hcount"].astype(np.int64)
    return out


@pytest.mark.parametrize("name,rows,walks", [
    ("lshape4096", [0, 1777, 4095], None),
    ("ball4096", [0, 2048, 4095], None),
    # the 3-D cube minus ball at its full site and node counts (tallies
    # written straight to HBM); 500 walks per site keep the oracle's
    # brute-force binning of the sampled rows short
    ("cubeball32768", [0, 32767], 500),
])
def test_full_size_fp32_sampled_rows(name, rows, walks):
    """The other configurations at their full sizes, in the launch shape the
    benchmark uses; the oracle recomputes sampled rows from the same
    streams, compared statistically as for the square."""
    c = W.config(name)
    N = walks or c["walks"]
    tb = _gpu_tb(c["domain"], c["sites"], c["bnodes"], N, c["eps"], c["seed"], precision="f32")
    info = tb.info()
    assert info["walks"] == len(c["sites"]) * N
    rows = np.array(rows)
    g = _export_rows(tb, rows)
    assert np.all(g["Hcount"].sum(axis=1) == N)
    bn = c["bnodes"]
    gb = bn[:, 0] ** 2 - bn[:, 1] ** 2          # harmonic in 2-D and 3-D
    _say("oracle rows", name, rows.tolist())
    ref = _oracle_rows_with_se(c["domain"], c["sites"], bn, N, c["eps"], c["seed"], rows, gb)
    _check_f32_rows(g, ref, np.arange(len(rows)), gb, _np(tb.export("site_steps"))[rows])
    del tb
    torch.cuda.empty_cache()


# ----------------------------------------------------------------- apply


def test_apply_matches_exported_matrices():
    dom = W.unit_disk()
    sites = W.sample_sites(dom, 70, 2, 1e-3)
    bn = W.circle_nodes(33)
    for prec in ("f64", "f32"):
        tb = _gpu_tb(dom, sites, bn, 500, 1e-3, 6, precision=prec, volume_samples=1 << 12)
        g = _export_all(tb)
        rng = np.random.default_rng(0)
        fbar = rng.normal(size=70)
        gg = rng.normal(size=33)
        u, gu = tb.apply(torch.tensor(fbar, device="cuda"), torch.tensor(gg, device="cuda"))
        torch.cuda.synchronize()
        A = g["A"].astype(np.float64)
        ref_u = A @ fbar + g["H"].astype(np.float64) @ gg
        ref_g = np.einsum("anm,m->an", g["B"].astype(np.float64), fbar) + \
            np.einsum("anp,p->an", g["K"].astype(np.float64), gg)
        assert np.allclose(_np(u), ref_u, rtol=1e-12, atol=1e-12)
        assert np.allclose(_np(gu), ref_g, rtol=1e-12, atol=1e-12)


def test_disk_poisson_direct_apply():
    """-Lap u = 1 on the unit disk: (1/2) A 1 -> (1 - |x|^2)/4 (accuracy)."""
    c = W.config("disk64")
    tb = _gpu_tb(c["domain"], c["sites"], c["bnodes"], 20000, c["eps"], 1, precision="f64",
                 volume_samples=1 << 12)
    u, _ = tb.apply(torch.full((64,), 0.5, dtype=torch.float64, device="cuda"),
                    torch.zeros(64, dtype=torch.float64, device="cuda"))
    exact = (1 - (c["sites"] ** 2).sum(1)) / 4
    assert np.abs(_np(u) - exact).max() < 0.01
