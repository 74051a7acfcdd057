"""Prepared solution operators (wos_operator_* and wos_server_submit_op)
against the oracle's Tikhonov solve and against wos_solve.

An operator is the linear map (f, g) -> u of one toolbox and one set of
coefficients, written out as dense matrices; applied to any data it must
give the solve's u and grad u to rounding (FP64 storage) or to FP32
rounding of the stored matrices (FP32 storage)."""
import ctypes
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


def _coeffs(x):
    """Anisotropic SPD A (up to 1:50), smooth b, c > 0 at the points x."""
    n = len(x)
    th = np.pi * x[:, 0]
    kap = 1.0 + 49.0 * (0.5 + 0.5 * np.sin(3 * x[:, 1]))
    R = np.stack([np.stack([np.cos(th), -np.sin(th)], -1), np.stack([np.sin(th), np.cos(th)], -1)], -2)
    A = R @ (np.eye(2)[None] * np.stack([np.ones(n), kap], -1)[:, None, :]) @ np.transpose(R, (0, 2, 1))
    b = 0.5 * np.stack([np.sin(2 * x[:, 1]), np.cos(x[:, 0])], 1)
    c = 0.2 + 0.0 * x[:, 0]
    return A, b, c


def _build(dom, sites, bn, walks, eps, precision, seed=11):
    _say("GPU build", dom["kind"], len(sites), len(bn), walks, precision)
    tb = P.Toolbox(dom, sites, bn, walks, eps, seed=seed, precision=precision, volume_samples=1 << 18)
    tb.build()
    torch.cuda.synchronize()
    mats = {k: tb.export(k).cpu().numpy().astype(np.float64) for k in ("A", "B", "H", "K", "lambda")}
    return tb, mats


def _data(tb, k, seed):
    rng = np.random.default_rng(seed)
    x, z = tb.sites, tb.bnodes
    f = np.stack([np.cos((1 + j) * x[:, 0]) + rng.normal(0, 0.1, tb.n) for j in range(k)])
    g = np.stack([z[:, 0] ** 2 - z[:, 1] ** 2 + rng.normal(0, 0.1, tb.p) for j in range(k)])
    return f, g


@pytest.fixture(scope="module")
def disk64():
    dom = W.unit_disk()
    sites = W.sample_sites(dom, 91, 3, 1e-2)
    return _build(dom, sites, W.circle_nodes(30), 1500, 1e-3, "f64")


@pytest.fixture(scope="module")
def square32():
    dom = W.unit_square()
    sites = W.sample_sites(dom, 300, 5, 1e-3)    # several panels of 64, ragged last one
    return _build(dom, sites, W.square_nodes(20), 1500, 1e-4, "f32")


@pytest.mark.parametrize("rcond", [1e-3, 1e-2])
def test_operator_matches_oracle_fp64(disk64, rcond):
    tb, mats = disk64
    lam = mats["lambda"]
    A, b, c = _coeffs(tb.sites)
    op = tb.operator(A=A, b=b, c=c, rcond=rcond, grad=True)
    info = op.info()
    _say("operator", info)
    f, g = _data(tb, 3, 1)
    u, gu = op.apply(f, g, grad=True)
    torch.cuda.synchronize()
    u, gu = u.cpu().numpy(), gu.cpu().numpy()
    for r in range(3):
        ref = OL.solve_linear(mats, lam, f[r], g[r], Acoef=A, bcoef=b, ccoef=c, rcond=rcond, solver="tikhonov")
        if r == 0:
            _, reg = OL.tikhonov_solve(ref["Lambda"], OL.rhs(mats, lam, ref["Sigma"], f[r], g[r]), rcond)
            assert np.isclose(info["reg"], reg, rtol=1e-10)
        assert _lam_rel(u[r], ref["u"], lam) < 1e-8
        scale = np.abs(ref["grad_u"]).max()
        assert np.allclose(gu[r], ref["grad_u"], rtol=1e-7, atol=1e-8 * scale)


def test_operator_matches_solve_on_fp32_toolbox(square32):
    """Against wos_solve (Tikhonov, FP64) on the same FP32 toolbox, for 11
    right-hand sides (a full batch of 8 and a ragged one of 3), FP64 and FP32
    storage, with and without the gradient."""
    tb, mats = square32
    lam = mats["lambda"]
    A, b, c = _coeffs(tb.sites)
    f, g = _data(tb, 11, 2)
    ref_u, ref_g = [], []
    for r in range(11):
        u, gu, _, _ = tb.solve(f[r], g[r], kind="linear", A=A, b=b, c=c, rcond=1e-3, solver="tikhonov")
        ref_u.append(u.cpu().numpy())
        ref_g.append(gu.cpu().numpy())
    op64 = tb.operator(A=A, b=b, c=c, rcond=1e-3, grad=True, storage="f64")
    op32 = tb.operator(A=A, b=b, c=c, rcond=1e-3, grad=False, storage="f32")
    assert op32.info()["device_bytes"] * 6 == op64.info()["device_bytes"]  # n rows of 4 B vs 3n rows of 8 B
    u64, g64 = op64.apply(f, g, grad=True)
    u64n, _ = op64.apply(f, g, grad=False)
    u32, _ = op32.apply(f, g)
    torch.cuda.synchronize()
    u64, g64, u64n, u32 = (t.cpu().numpy() for t in (u64, g64, u64n, u32))
    assert np.array_equal(u64, u64n) or np.allclose(u64, u64n, rtol=1e-13, atol=1e-15)
    for r in range(11):
        assert _lam_rel(u64[r], ref_u[r], lam) < 1e-8
        scale = np.abs(ref_g[r]).max()
        assert np.allclose(g64[r], ref_g[r], rtol=1e-7, atol=1e-8 * scale)
        # FP32 storage: each product sums n + p terms of relative error 2^-24
        assert _lam_rel(u32[r], ref_u[r], lam) < 2e-6
    # one right-hand side at a time gives the batched result
    for r in (0, 7, 10):
        u1, _ = op64.apply(f[r], g[r])
        assert np.allclose(u1.cpu().numpy(), u64[r], rtol=1e-13, atol=1e-14 * np.abs(u64[r]).max())


def test_operator_errors(disk64):
    tb, _ = disk64
    zf = torch.zeros(tb.n, dtype=torch.float64, device="cuda")
    zg = torch.zeros(tb.p, dtype=torch.float64, device="cuda")
    opts = P._lib.WosOperatorOpts(want_grad=0, storage=1)
    for kw, status in ((dict(kind="linear", solver="tsvd"), "ENOTIMPL"),
                       (dict(kind="quasilinear", solver="tikhonov"), "EINVAL")):
        _, _, _, _, _, co = tb._coeffs(zf, zg, **kw)
        h = ctypes.c_void_p()
        with pytest.raises(P.WosError, match=status):
            P._lib.check(P._lib.lib().wos_operator_create(tb._h, ctypes.byref(co), ctypes.byref(opts), None,
                                                          ctypes.byref(h)))
        assert not h.value
    op = tb.operator(rcond=1e-2, grad=False)
    f, g = _data(tb, 1, 3)
    with pytest.raises(P.WosError, match="EINVAL"):
        op.apply(f, g, grad=True)


def test_served_operator_requests_batch_and_match(disk64):
    """Operator requests queued together are solved as batches; every result
    equals the operator applied alone, with plain solves in the same mix."""
    tb, mats = disk64
    A, b, c = _coeffs(tb.sites)
    op = tb.operator(A=A, b=b, c=c, rcond=1e-2, grad=True)
    f, g = _data(tb, 20, 4)
    alone = [op.apply(f[r], g[r], grad=True) for r in range(20)]
    plain_alone = tb.solve(f[0], g[0], kind="linear", A=A, b=b, c=c, rcond=1e-2, solver="tikhonov")[0]
    torch.cuda.synchronize()
    sv = P.Server(slots=3, max_batch=6)
    tickets = []
    for r in range(20):
        tickets.append(("op", r) + sv.submit_op(op, f[r], g[r], grad=(r % 2 == 0)))
        if r % 7 == 3:
            tickets.append(("plain", r) + sv.submit(tb, f[0], g[0], kind="linear", A=A, b=b, c=c, rcond=1e-2,
                                                   solver="tikhonov"))
    for kind, r, t, u, gu in tickets:
        sv.poll(t)
        if kind == "op":
            ua, ga = alone[r]
            assert np.allclose(u.cpu().numpy(), ua.cpu().numpy(), rtol=1e-12, atol=1e-14)
            if gu is not None:
                assert np.allclose(gu.cpu().numpy(), ga.cpu().numpy(), rtol=1e-12, atol=1e-13)
        else:
            assert np.allclose(u.cpu().numpy(), plain_alone.cpu().numpy(), rtol=1e-9, atol=1e-12)
    sv.close()
