"""Solve path on the GPU (wos_solve through the C ABI) against the oracle.

The GPU toolbox is exported and handed to the oracle's assembly and
truncated-SVD solve (FP64, numpy SVD), so both sides solve the same
system; they must agree to rounding.  The truncation keeps the same
singular values on both sides only if none sits at the threshold: each case
checks the gap first.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import linalg as OL

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2608_07017_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rings(K):
    pts = []
    for k in range(1, K + 1):
        nk = 6 * k - 3
        r = (k - 0.5) / K
        th = 2 * np.pi * np.arange(nk) / nk
        pts.append(np.stack([r * np.cos(th), r * np.sin(th)], 1))
    return np.concatenate(pts)


def _build(dom, sites, bn, walks, eps, precision="f64", seed=11):
    _say("GPU build", dom["kind"], len(sites), len(bn), walks, precision)
    tb = P.Toolbox(dom, sites, bn, walks, eps, seed=seed, precision=precision, volume_samples=1 << 18)
    tb.build()
    torch.cuda.synchronize()
    mats = {k: tb.export(k).cpu().numpy().astype(np.float64) for k in ("A", "B", "H", "K", "lambda")}
    return tb, mats


def _lam_rel(u, v, lam):
    return np.sqrt(np.sum(lam * (u - v) ** 2)) / np.sqrt(np.sum(lam * v ** 2))


def _safe_rcond(M, candidates=(1e-3, 2e-3, 5e-3, 1e-2, 3e-2)):
    s = np.linalg.svd(M, compute_uv=False)
    for rc in candidates:
        thr = rc * s[0]
        if np.min(np.abs(s - thr)) > 1e-4 * thr:
            return rc, int(np.sum(s > thr))
    pytest.skip("every candidate threshold sits on a singular value")


@pytest.fixture(scope="module")
def disk_tb():
    dom = W.unit_disk()
    sites = _rings(5)
    return _build(dom, sites, W.circle_nodes(30), 1500, 1e-3)


def test_linear_laplace_symmetric(disk_tb):
    tb, mats = disk_tb
    n = tb.n
    lam = mats["lambda"]
    f = -np.ones(n)          # paper's convention: Lap u = -1
    g = np.zeros(tb.p)
    Lam, Sig = OL.assemble(mats, lam)
    rc, rank = _safe_rcond(Lam)
    ref = OL.solve_linear(mats, lam, f, g, rcond=rc)
    u, gu, q, info = tb.solve(f, g, kind="linear", rcond=rc)
    torch.cuda.synchronize()
    assert info["rank"] == rank
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-9
    assert np.allclose(gu.cpu().numpy(), ref["grad_u"], rtol=1e-7, atol=1e-9)
    # the system itself: Lambda q = rhs on the kept subspace
    assert np.isclose(info["sigma_max"], np.linalg.svd(Lam, compute_uv=False)[0], rtol=1e-10)


def test_linear_anisotropic_reaction_symmetric(disk_tb):
    tb, mats = disk_tb
    n = tb.n
    lam = mats["lambda"]
    rng = np.random.default_rng(3)
    x = _rings(5)
    th = np.pi * x[:, 0]
    kap = 1.0 + 9.0 * (0.5 + 0.5 * np.sin(3 * x[:, 1]))
    R = np.stack([np.stack([np.cos(th), -np.sin(th)], -1), np.stack([np.sin(th), np.cos(th)], -1)], -2)
    A = R @ (np.eye(2)[None] * np.stack([np.ones(n), kap], -1)[:, None, :]) @ np.transpose(R, (0, 2, 1))
    c = 0.5 + rng.random(n)
    f = np.cos(2 * x[:, 0]) + x[:, 1]
    g = np.sin(np.arctan2(*W.circle_nodes(30).T[::-1]))
    Lam, Sig = OL.assemble(mats, lam, A, None, c)
    rc, rank = _safe_rcond(Lam)
    ref = OL.solve_linear(mats, lam, f, g, Acoef=A, ccoef=c, rcond=rc)
    u, gu, q, info = tb.solve(f, g, kind="linear", A=A, c=c, rcond=rc)
    torch.cuda.synchronize()
    assert info["rank"] == rank
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-9


def test_linear_advection_nonsymmetric(disk_tb):
    tb, mats = disk_tb
    n = tb.n
    lam = mats["lambda"]
    x = _rings(5)
    b = np.stack([-x[:, 1], x[:, 0]], 1)       # the paper's Ex. elliptic-div drift
    A = np.stack([np.stack([2 + x[:, 0] ** 2, x[:, 0] * x[:, 1]], -1),
                  np.stack([x[:, 0] * x[:, 1], 2 + x[:, 1] ** 2], -1)], -2)
    c = np.ones(n)
    f = np.sin(np.pi * x[:, 0])
    g = np.zeros(tb.p)
    Lam, Sig = OL.assemble(mats, lam, A, b, c)
    rc, rank = _safe_rcond(Lam)
    ref = OL.solve_linear(mats, lam, f, g, Acoef=A, bcoef=b, ccoef=c, rcond=rc)
    u, gu, q, info = tb.solve(f, g, kind="linear", A=A, b=b, c=c, rcond=rc)
    torch.cuda.synchronize()
    assert info["rank"] == rank
    # the right singular vectors come from Lambda^T Lambda: cond^2 rounding
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-7


def test_newton_semilinear_cubic(disk_tb):
    # The truncated directions keep a gradient component that Newton cannot
    # remove, so the iteration is compared at a fixed count (tol never met).
    tb, mats = disk_tb
    lam = mats["lambda"]
    x = _rings(5)
    ue, ge, le = W.smooth_field(7, 2, terms=4, max_freq=2.0, scale=0.5)
    f = -le(x) + ue(x) ** 3
    g = ue(W.circle_nodes(30))
    Lam0, _ = OL.assemble(mats, lam)
    rc, _ = _safe_rcond(Lam0, (1e-2, 2e-2, 3e-2, 5e-2))
    ref = OL.newton_cubic(mats, lam, f, g, kappa=1.0, rcond=rc, tol=1e-300, max_iter=6)
    u, gu, q, info = tb.solve(f, g, kind="semilinear_cubic", kappa=1.0, rcond=rc, tol=1e-300, max_iter=6)
    torch.cuda.synchronize()
    assert info["iters"] == ref["iters"] == 6
    assert np.isclose(info["grad_norm0"], ref["grad_norm0"], rtol=1e-8)
    assert np.isclose(info["grad_norm"], ref["grad_norm"], rtol=1e-6)
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-8
    assert np.allclose(q.cpu().numpy(), ref["h"], rtol=1e-6, atol=1e-8 * np.abs(ref["h"]).max())


def test_picard_quasilinear(disk_tb):
    tb, mats = disk_tb
    lam = mats["lambda"]
    x = _rings(5)
    f = 2.0 + x[:, 0]
    g = 0.2 * W.circle_nodes(30)[:, 1]
    Lam0, _ = OL.assemble(mats, lam)
    rc, _ = _safe_rcond(Lam0, (1e-2, 2e-2, 3e-2, 5e-2))
    # the update ratio falls by about 10x per sweep here: tol = 1e-9 is met
    # after a handful of sweeps on both sides, far from any crossing
    ref = OL.picard_quasilinear(mats, lam, f, g, rcond=rc, tol=1e-9, max_iter=60)
    u, gu, q, info = tb.solve(f, g, kind="quasilinear", rcond=rc, tol=1e-9, max_iter=60)
    torch.cuda.synchronize()
    assert 2 < ref["iters"] < 60
    assert info["iters"] == ref["iters"]
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-8
    # fixed sweep count, tolerance never met
    ref = OL.picard_quasilinear(mats, lam, f, g, rcond=rc, tol=1e-300, max_iter=4)
    u, gu, q, info = tb.solve(f, g, kind="quasilinear", rcond=rc, tol=1e-300, max_iter=4)
    torch.cuda.synchronize()
    assert info["iters"] == ref["iters"] == 4
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-8


def test_fp32_toolbox_square_linear():
    dom = W.unit_square()
    sites, bn = W.paper_square_layout()
    sites = sites[::4]                 # 100 cell centres, ragged against 64-wide tiles
    tb, mats = _build(dom, sites, bn, 2000, 1e-4, precision="f32")
    lam = mats["lambda"]
    f = np.ones(len(sites))
    g = bn[:, 0] ** 2 - bn[:, 1] ** 2
    Lam, _ = OL.assemble(mats, lam)
    rc, rank = _safe_rcond(Lam)
    ref = OL.solve_linear(mats, lam, f, g, rcond=rc)
    u, gu, q, info = tb.solve(f, g, kind="linear", rcond=rc)
    torch.cuda.synchronize()
    assert info["rank"] == rank
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-9


def test_solve_rejects_bad_input(disk_tb):
    tb, _ = disk_tb
    with pytest.raises(P.WosError):
        tb.solve(np.zeros(tb.n), np.zeros(tb.p), kind="linear", rcond=2.0)


# ---------------------------------------------------------------- Tikhonov
def _tik_problem(x, n, d):
    th = np.pi * x[:, 0]
    kap = 1.0 + 49.0 * (0.5 + 0.5 * np.sin(3 * x[:, 1]))
    R = np.stack([np.stack([np.cos(th), -np.sin(th)], -1), np.stack([np.sin(th), np.cos(th)], -1)], -2)
    A = R @ (np.eye(2)[None] * np.stack([np.ones(n), kap], -1)[:, None, :]) @ np.transpose(R, (0, 2, 1))
    b = 0.5 * np.stack([np.sin(2 * x[:, 1]), np.cos(x[:, 0])], 1)
    c = 0.2 + 0.0 * x[:, 0]
    return A, b, c


@pytest.mark.parametrize("rcond", [1e-3, 1e-2])
def test_tikhonov_f64_matches_oracle(disk_tb, rcond):
    tb, mats = disk_tb
    n = tb.n
    lam = mats["lambda"]
    x = _rings(5)
    A, b, c = _tik_problem(x, n, 2)
    f = np.cos(2 * x[:, 0]) + x[:, 1]
    g = 0.3 * W.circle_nodes(30)[:, 0]
    ref = OL.solve_linear(mats, lam, f, g, Acoef=A, bcoef=b, ccoef=c, rcond=rcond, solver="tikhonov")
    _, reg = OL.tikhonov_solve(ref["Lambda"], OL.rhs(mats, lam, ref["Sigma"], f, g), rcond)
    u, gu, q, info = tb.solve(f, g, kind="linear", A=A, b=b, c=c, rcond=rcond, solver="tikhonov")
    torch.cuda.synchronize()
    assert np.isclose(info["reg"], reg, rtol=1e-10)
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-9
    assert np.allclose(q.cpu().numpy(), ref["q"], rtol=1e-7, atol=1e-9 * np.abs(ref["q"]).max())


@pytest.fixture(scope="module")
def square_f32_tb():
    dom = W.unit_square()
    sites = W.sample_sites(dom, 300, 5, 1e-3)    # several Cholesky panels, ragged last one
    bn = W.square_nodes(20)
    return _build(dom, sites, bn, 1500, 1e-4, precision="f32")


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_tikhonov_on_fp32_toolbox_matches_oracle(square_f32_tb, precision):
    tb, mats = square_f32_tb
    n = tb.n
    lam = mats["lambda"]
    x = tb.sites
    A, b, c = _tik_problem(x, n, 2)
    f = np.sin(np.pi * x[:, 0]) * (1 + x[:, 1])
    bn = tb.bnodes
    g = bn[:, 0] ** 2 - bn[:, 1] ** 2
    ref = OL.solve_linear(mats, lam, f, g, Acoef=A, bcoef=b, ccoef=c, rcond=1e-3, solver="tikhonov")
    u, gu, q, info = tb.solve(f, g, kind="linear", A=A, b=b, c=c, rcond=1e-3, solver="tikhonov",
                              precision=precision, refine_tol=1e-13, max_refine=30)
    torch.cuda.synchronize()
    _say(precision, info)
    _, reg = OL.tikhonov_solve(ref["Lambda"], OL.rhs(mats, lam, ref["Sigma"], f, g), 1e-3)
    # both routes take reg from exact FP64 columns of Lambda
    assert np.isclose(info["reg"], reg, rtol=1e-12)
    if precision == "mixed":
        assert info["fallback"] == 0 and info["refine_converged"] == 1
        assert info["refine_iters"] >= 1 and info["refine_residual"] <= 1e-13
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-9


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_tikhonov_many_panels_matches_oracle(precision):
    """1100 sites: the Cholesky factorisation runs over 18 panels of 64 (the
    last one ragged) and the triangular inverse recurses five levels."""
    dom = W.unit_square()
    sites = W.sample_sites(dom, 1100, 9, 1e-3)
    tb, mats = _build(dom, sites, W.square_nodes(32), 400, 1e-3, precision="f32")
    lam = mats["lambda"]
    A, b, c = _tik_problem(sites, len(sites), 2)
    f = np.sin(np.pi * sites[:, 0]) * (1 + sites[:, 1])
    g = tb.bnodes[:, 0] ** 2 - tb.bnodes[:, 1] ** 2
    ref = OL.solve_linear(mats, lam, f, g, Acoef=A, bcoef=b, ccoef=c, rcond=1e-2, solver="tikhonov")
    u, gu, q, info = tb.solve(f, g, kind="linear", A=A, b=b, c=c, rcond=1e-2, solver="tikhonov",
                              precision=precision, refine_tol=1e-13, max_refine=30)
    torch.cuda.synchronize()
    _say("many panels", precision, info)
    assert info["fallback"] == 0 and info["refine_converged"] == 1
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-9


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_newton_tikhonov_matches_oracle(square_f32_tb, precision):
    tb, mats = square_f32_tb
    lam = mats["lambda"]
    x = tb.sites
    ue, ge, le = W.smooth_field(7, 2, terms=4, max_freq=2.0, scale=0.5)
    f = -le(x) + ue(x) ** 3
    g = ue(tb.bnodes)
    ref = OL.newton_cubic(mats, lam, f, g, kappa=1.0, rcond=1e-2, tol=1e-300, max_iter=5, solver="tikhonov")
    u, gu, q, info = tb.solve(f, g, kind="semilinear_cubic", kappa=1.0, rcond=1e-2, tol=1e-300, max_iter=5,
                              solver="tikhonov", precision=precision, refine_tol=1e-13, max_refine=30)
    torch.cuda.synchronize()
    _say("newton", precision, info)
    assert info["iters"] == ref["iters"] == 5
    assert info["refine_converged"] == 1
    assert np.isclose(info["grad_norm0"], ref["grad_norm0"], rtol=1e-6)
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-9


def test_picard_tikhonov_matches_oracle(disk_tb):
    tb, mats = disk_tb
    lam = mats["lambda"]
    x = _rings(5)
    f = 2.0 + x[:, 0]
    g = 0.2 * W.circle_nodes(30)[:, 1]
    ref = OL.picard_quasilinear(mats, lam, f, g, rcond=3e-2, tol=1e-300, max_iter=4, solver="tikhonov")
    u, gu, q, info = tb.solve(f, g, kind="quasilinear", rcond=3e-2, tol=1e-300, max_iter=4, solver="tikhonov")
    torch.cuda.synchronize()
    assert info["iters"] == ref["iters"] == 4
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-9


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_tikhonov_4096_sites_wide_tiles(precision):
    """4096 sites: the products that form Lambda (4096 x 4096 from 3 x 4096
    rows) and the normal matrix take the 128 x 128 tiles of the matrix-core
    GEMM (at least 256 tiles of 128), FP64 and FP32, against the oracle's
    FP64 solve on the same exported toolbox.  The mixed route's FP32 factor
    is only a preconditioner, so few refinement steps also vouch for the
    FP32 tiles."""
    dom = W.unit_square()
    sites = W.sample_sites(dom, 4096, 12, 1e-3)
    tb, mats = _build(dom, sites, W.square_nodes(64), 200, 1e-3, precision="f32")
    lam = mats["lambda"]
    A, b, c = _tik_problem(sites, len(sites), 2)
    f = np.sin(np.pi * sites[:, 0]) * (1 + sites[:, 1])
    g = tb.bnodes[:, 0] ** 2 - tb.bnodes[:, 1] ** 2
    _say("oracle Tikhonov, 4096 sites")
    ref = OL.solve_linear(mats, lam, f, g, Acoef=A, bcoef=b, ccoef=c, rcond=1e-2, solver="tikhonov")
    u, gu, q, info = tb.solve(f, g, kind="linear", A=A, b=b, c=c, rcond=1e-2, solver="tikhonov",
                              precision=precision, refine_tol=1e-13, max_refine=30)
    torch.cuda.synchronize()
    _say("4096", precision, info)
    assert info["fallback"] == 0 and info["refine_converged"] == 1
    if precision == "mixed":
        assert info["refine_iters"] <= 8
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-9
    # the first FP32 product of each shape class times both tilings (and
    # keeps the faster); the tilings add in the same order, so a second
    # solve, on the kept tiling, gives the same bits
    u2, _, _, info2 = tb.solve(f, g, kind="linear", A=A, b=b, c=c, rcond=1e-2, solver="tikhonov",
                               precision=precision, refine_tol=1e-13, max_refine=30)
    torch.cuda.synchronize()
    assert torch.equal(u, u2) and info2["refine_iters"] == info["refine_iters"]


def test_paper_elliptic_div_example_end_to_end():
    """The example "elliptic div" end to end on the paper's disk layout
    (300 ring sites, 60 boundary nodes, M = 30 steps per walk): A(x) =
    [[2 + x^2, xy], [xy, 2 + y^2]], b = (-y, x), c = 1, u = (1 - |x|^2)
    sin(pi x), solved through eq. linear_q by the truncated SVD with
    rcond 1e-3 (Table "numerical parameters").  The GPU solve against the
    oracle's on the same matrices; the singular values of Lambda in the
    range the paper notes (sigma_max about 1e-2, sigma_min about 1e-7); the
    L^2 error near the layout's discretisation floor (8.5e-2)."""
    dom = W.unit_disk()
    sites, bn = W.paper_disk_layout()
    _say("GPU build: paper disk layout, 1e5 walks, M = 30")
    tb = P.Toolbox(dom, sites, bn, 100_000, 0.0, seed=7, precision="f64", fixed_M=30, volume_samples=1 << 22)
    tb.build()
    torch.cuda.synchronize()
    mats = {k: tb.export(k).cpu().numpy() for k in ("A", "B", "H", "K", "lambda")}
    lam = mats["lambda"]
    uex, guex, f = W.elliptic_div_disk(sites)
    A, b, c = W.elliptic_div_coef(sites)
    g = np.zeros(len(bn))
    u, gu, q, info = tb.solve(f, g, kind="linear", A=A, b=b, c=c, rcond=1e-3, solver="tsvd")
    torch.cuda.synchronize()
    u = u.cpu().numpy()
    Lam, _ = OL.assemble(mats, lam, A, b, c)
    s = np.linalg.svd(Lam, compute_uv=False)
    _say("sigma_max %.3e sigma_min %.3e rank %d" % (s[0], s[-1], info["rank"]))
    assert np.isclose(info["sigma_max"], s[0], rtol=1e-9)
    assert 2e-3 < s[0] < 5e-2 and 1e-9 < s[-1] < 1e-5
    ref = OL.solve_linear(mats, lam, f, g, Acoef=A, bcoef=b, ccoef=c, rcond=1e-3)
    if np.min(np.abs(s - 1e-3 * s[0])) > 1e-4 * 1e-3 * s[0]:
        assert info["rank"] == int(np.sum(s > 1e-3 * s[0]))
        assert _lam_rel(u, ref["u"], lam) < 1e-7
    err = W.voronoi_l2_error(dom, sites, u, lambda x: W.elliptic_div_disk(x)[0], npoints=1 << 21)
    site_rms = np.sqrt(np.sum(lam * (u - uex) ** 2))
    _say("L2 error %.4f (floor 0.0853), lambda-weighted site RMS %.4f" % (err, site_rms))
    assert err < 0.11
