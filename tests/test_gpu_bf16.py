"""BF16 route on the GPU: the toolbox's BF16 shadows, the matrix-core BF16
product, the BF16 apply and the BF16-preconditioned solve (include/wos.h:
wos_toolbox_make_bf16, wos_gemm_bf16_nt, wos_apply_bf16,
WOS_SOLVE_MIXED_BF16).

The shadows must be the toolbox rounded to nearest even, bit for bit; the
product and the apply must equal FP64 products of the BF16 values to their
accumulation rounding; the solve must reach the FP64 route's solution of
the same regularised system (the BF16 factor is a preconditioner only), and
the unrefined BF16 apply error against the FP32 toolbox is stated."""
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


def _lam_rel(u, v, lam):
    return np.sqrt(np.sum(lam * (u - v) ** 2)) / np.sqrt(np.sum(lam * v ** 2))


@pytest.mark.parametrize("M,N,K,ragged", [(300, 257, 1003, False), (512, 512, 4096, False), (129, 1, 40, False),
                                          (200, 130, 77, True)])
def test_gemm_bf16_nt_matches_fp64(M, N, K, ragged):
    g = torch.Generator().manual_seed(M + N + K)
    if ragged:   # rows not 16-byte aligned: the element-load path
        Xb = torch.randn(M, K + 3, generator=g).bfloat16()[:, 1:K + 1]
        Yb = torch.randn(N, K + 5, generator=g).bfloat16()[:, 2:K + 2]
    else:
        Xb = torch.randn(M, K, generator=g).bfloat16()
        Yb = torch.randn(N, K, generator=g).bfloat16()
    C0 = torch.randn(M, N, generator=g)
    _say("gemm bf16", M, N, K, "ragged" if ragged else "")
    Xd, Yd = Xb.cuda(), Yb.cuda()
    C = P.gemm_bf16_nt(Xd, Yd)
    C2 = P.gemm_bf16_nt(Xd, Yd, C=C0.clone().cuda(), alpha=0.5, beta=2.0)
    torch.cuda.synchronize()
    ref = Xb.double() @ Yb.double().T
    scale = Xb.double().abs() @ Yb.double().abs().T
    assert torch.all((C.cpu().double() - ref).abs() <= 1e-5 * scale + 1e-30)
    ref2 = 0.5 * ref + 2.0 * C0.double()
    assert torch.all((C2.cpu().double() - ref2).abs() <= 1e-5 * (0.5 * scale + 2.0 * C0.double().abs()) + 1e-30)


@pytest.mark.parametrize("ragged", [False, True])
def test_gemm_bf16_nt_large_tiles(ragged):
    # at least one 256 x 256 tile per compute unit: the large-tile kernel,
    # ragged in both sides; its leading block must equal, bit for bit, the
    # product of the leading rows alone (the 128 x 128 kernel): every element
    # adds the same products in the same order
    M, N, K = 4100, 4097, 200
    g = torch.Generator().manual_seed(5 + ragged)
    if ragged:
        Xb = torch.randn(M, K + 3, generator=g).bfloat16()[:, 1:K + 1]
        Yb = torch.randn(N, K + 5, generator=g).bfloat16()[:, 2:K + 2]
    else:
        Xb = torch.randn(M, K, generator=g).bfloat16()
        Yb = torch.randn(N, K, generator=g).bfloat16()
    _say("gemm bf16 large tiles", M, N, K, "ragged" if ragged else "")
    Xd, Yd = Xb.cuda(), Yb.cuda()
    C = P.gemm_bf16_nt(Xd, Yd)
    Cs = P.gemm_bf16_nt(Xd[:300], Yd[:260])
    torch.cuda.synchronize()
    ref = Xb.double() @ Yb.double().T
    scale = Xb.double().abs() @ Yb.double().abs().T
    assert torch.all((C.cpu().double() - ref).abs() <= 1e-5 * scale + 1e-30)
    assert torch.equal(C[:300, :260].cpu(), Cs.cpu())


@pytest.fixture(scope="module")
def square_tb():
    dom = W.unit_square()
    sites = W.sample_sites(dom, 300, 5, 1e-3)
    bn = W.square_nodes(20)
    _say("GPU build: square 300 sites FP32")
    tb = P.Toolbox(dom, sites, bn, 1500, 1e-4, seed=11, precision="f32", volume_samples=1 << 18)
    tb.build()
    torch.cuda.synchronize()
    mats = {k: tb.export(k).cpu().numpy().astype(np.float64) for k in ("A", "B", "H", "K", "lambda")}
    return tb, mats


def _expected_shadows(tb):
    d, n = tb.dim, tb.n
    A, B, H, K = (tb.export(k).cpu() for k in ("A", "B", "H", "K"))
    LV = torch.cat([B.reshape(d * n, -1), A], 0).T.contiguous()   # m x (d+1) n
    LG = torch.cat([K.reshape(d * n, -1), H], 0).T.contiguous()
    return LV.bfloat16().view(torch.int16), LG.bfloat16().view(torch.int16)


def test_shadows_are_the_rounded_toolbox(square_tb):
    tb, _ = square_tb
    tb.make_bf16()
    torch.cuda.synchronize()
    ev, eg = _expected_shadows(tb)
    assert torch.equal(tb.export("shadow_v").cpu(), ev)
    assert torch.equal(tb.export("shadow_g").cpu(), eg)


def test_apply_bf16(square_tb):
    tb, mats = square_tb
    rng = np.random.default_rng(2)
    fbar = rng.normal(size=tb.m)
    g = tb.bnodes[:, 0] ** 2 - tb.bnodes[:, 1] ** 2
    u, gu = tb.apply_bf16(fbar, g)
    u32, gu32 = tb.apply(fbar, g)
    torch.cuda.synchronize()
    # the product of the BF16 values, in FP64
    SV = tb.export("shadow_v").cpu().view(torch.bfloat16).double().numpy()
    SG = tb.export("shadow_g").cpu().view(torch.bfloat16).double().numpy()
    y = SV.T @ fbar + SG.T @ g
    mag = np.abs(SV.T) @ np.abs(fbar) + np.abs(SG.T) @ np.abs(g)
    n, d = tb.n, tb.dim
    got = np.concatenate([gu.cpu().numpy().reshape(-1), u.cpu().numpy()])
    assert np.all(np.abs(got - y) <= 1e-13 * mag + 1e-300)
    # against the FP32 toolbox: the rounding of the toolbox to BF16 (2^-9
    # relative per entry, partly cancelling over a row); stated, and bounded
    err_u = np.abs(u.cpu().numpy() - u32.cpu().numpy()) / mag[d * n:]
    err_g = np.abs(gu.cpu().numpy() - gu32.cpu().numpy()).reshape(-1) / mag[:d * n]
    _say("BF16 apply relative error: u max %.2e, grad u max %.2e" % (err_u.max(), err_g.max()))
    assert err_u.max() <= 2.0 ** -8 and err_g.max() <= 2.0 ** -8


@pytest.mark.parametrize("rcond", [1e-3, 1e-2])
def test_solve_bf16_reaches_the_fp64_solution(square_tb, rcond):
    tb, mats = square_tb
    lam = mats["lambda"]
    x = tb.sites
    th = np.pi * x[:, 0]
    kap = 1.0 + 49.0 * (0.5 + 0.5 * np.sin(3 * x[:, 1]))
    R = np.stack([np.stack([np.cos(th), -np.sin(th)], -1), np.stack([np.sin(th), np.cos(th)], -1)], -2)
    A = R @ (np.eye(2)[None] * np.stack([np.ones(tb.n), kap], -1)[:, None, :]) @ np.transpose(R, (0, 2, 1))
    b = 0.5 * np.stack([np.sin(2 * x[:, 1]), np.cos(x[:, 0])], 1)
    c = 0.2 + 0.0 * x[:, 0]
    f = np.sin(np.pi * x[:, 0]) * (1 + x[:, 1])
    g = tb.bnodes[:, 0] ** 2 - tb.bnodes[:, 1] ** 2
    ref = OL.solve_linear(mats, lam, f, g, Acoef=A, bcoef=b, ccoef=c, rcond=rcond, solver="tikhonov")
    _, reg = OL.tikhonov_solve(ref["Lambda"], OL.rhs(mats, lam, ref["Sigma"], f, g), rcond)
    u, gu, q, info = tb.solve(f, g, kind="linear", A=A, b=b, c=c, rcond=rcond, solver="tikhonov", precision="bf16",
                              refine_tol=1e-13, max_refine=200)
    u64, _, _, _ = tb.solve(f, g, kind="linear", A=A, b=b, c=c, rcond=rcond, solver="tikhonov", precision="f64")
    torch.cuda.synchronize()
    _say("bf16 solve rcond %g:" % rcond, {k: info[k] for k in ("refine_iters", "refine_residual", "fallback")})
    assert info["fallback"] == 0 and info["refine_converged"] == 1
    assert np.isclose(info["reg"], reg, rtol=1e-12)
    assert _lam_rel(u.cpu().numpy(), u64.cpu().numpy(), lam) < 1e-9
    assert _lam_rel(u.cpu().numpy(), ref["u"], lam) < 1e-9


def test_picard_bf16_matches_f64(square_tb):
    tb, mats = square_tb
    lam = mats["lambda"]
    x = tb.sites
    f = 2.0 + x[:, 0]
    g = 0.2 * tb.bnodes[:, 1]
    kw = dict(kind="quasilinear", rcond=3e-2, tol=1e-300, max_iter=4, solver="tikhonov")
    u64, _, _, i64 = tb.solve(f, g, precision="f64", **kw)
    ubf, _, _, ibf = tb.solve(f, g, precision="bf16", refine_tol=1e-13, max_refine=200, **kw)
    torch.cuda.synchronize()
    assert ibf["iters"] == i64["iters"] == 4
    assert _lam_rel(ubf.cpu().numpy(), u64.cpu().numpy(), lam) < 1e-9


def test_shadows_follow_a_rebuild():
    dom = W.unit_disk()
    sites = W.sample_sites(dom, 64, 3, 1e-3)
    bn = W.circle_nodes(16)
    tb = P.Toolbox(dom, sites, bn, 300, 1e-3, seed=1, precision="f32", volume_samples=1 << 12).build()
    tb.make_bf16()
    tb.build(seed=2)           # the shadows of seed 1 are now stale
    fbar = np.linspace(-1, 1, tb.m)
    g = np.cos(np.arange(tb.p))
    u, _ = tb.apply_bf16(fbar, g)  # remakes them first
    torch.cuda.synchronize()
    ev, _ = _expected_shadows(tb)
    assert torch.equal(tb.export("shadow_v").cpu(), ev)
    SV = ev.view(torch.bfloat16).double().numpy()
    _, eg = _expected_shadows(tb)
    SG = eg.view(torch.bfloat16).double().numpy()
    y = SV.T @ fbar + SG.T @ g
    assert np.allclose(u.cpu().numpy(), y[tb.dim * tb.n:], rtol=1e-12, atol=1e-14)
    with pytest.raises(P.WosError):
        tb.solve(np.ones(tb.n), g, kind="semilinear_cubic", solver="tikhonov", precision="bf16")
