"""wos_solve_noalloc (the FP64 Tikhonov linear solve with the library's
fixed work array, for callers that cannot allocate) against wos_solve on the
same toolbox: the same bits, on two calls in a row, the second with a
smaller problem (the array keeps the first call's contents), and a problem
too large for the array refused before any launch."""
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2608_07017_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(sites, bn):
    x = sites
    th = 0.7 * np.sin(2 * x[:, 0] + x[:, 1])
    c, s = np.cos(th), np.sin(th)
    R = np.stack([np.stack([c, -s], -1), np.stack([s, c], -1)], -2)
    kap = 1.0 + 9.0 * (0.5 + 0.5 * np.cos(3 * x[:, 1]))
    A = R @ (np.eye(2)[None] * np.stack([np.ones(len(x)), kap], -1)[:, None, :]) @ np.transpose(R, (0, 2, 1))
    b = 0.5 * np.stack([np.sin(2 * x[:, 1]), np.cos(x[:, 0])], 1)
    f = np.sin(np.pi * x[:, 0]) * (1 + x[:, 1])
    g = bn[:, 0] ** 2 - bn[:, 1] ** 2
    return A, b, f, g


def _toolbox(n, seed):
    dom = W.unit_square()
    sites = W.sample_sites(dom, n, seed, 1e-3)
    bn = W.square_nodes(n // 12)
    _say("GPU build square n=%d p=%d" % (n, len(bn)))
    tb = P.Toolbox(dom, sites, bn, 400, 1e-4, seed=seed, precision="f32", volume_samples=1 << 16)
    tb.build()
    torch.cuda.synchronize()
    return tb, sites, bn


def _both(tb, sites, bn, rcond):
    A, b, f, g = _problem(sites, bn)
    u, gu, q, info = tb.solve(f, g, kind="linear", A=A, b=b, rcond=rcond, solver="tikhonov", precision="f64")
    u2 = torch.full((tb.n,), float("nan"), dtype=torch.float64, device="cuda")
    gu2 = torch.full((tb.dim, tb.n), float("nan"), dtype=torch.float64, device="cuda")
    q2 = torch.full((tb.m,), float("nan"), dtype=torch.float64, device="cuda")
    info2 = tb.solve_noalloc(f, g, u2, gu2, q2, A=A, b=b, rcond=rcond)
    torch.cuda.synchronize()
    return (u, gu, q, info), (u2, gu2, q2, info2)


def test_noalloc_solve_matches_wos_solve_on_two_calls():
    tb1, s1, b1 = _toolbox(600, 3)
    tb2, s2, b2 = _toolbox(240, 4)
    for tb, sites, bn, rcond in ((tb1, s1, b1, 1e-3), (tb2, s2, b2, 1e-2)):
        _say("noalloc vs solve, n=%d" % tb.n)
        (u, gu, q, info), (u2, gu2, q2, info2) = _both(tb, sites, bn, rcond)
        assert info2["reg"] == info["reg"]
        # the same kernels with fixed-order reductions: the same bits
        assert torch.equal(u2, u) and torch.equal(gu2, gu) and torch.equal(q2, q)
    tb1.free()
    tb2.free()


def test_noalloc_refuses_a_problem_beyond_its_array():
    tb, sites, bn = _toolbox(2400, 5)
    A, b, f, g = _problem(sites, bn)
    u = torch.zeros(tb.n, dtype=torch.float64, device="cuda")
    with pytest.raises(P.WosError) as e:
        tb.solve_noalloc(f, g, u, None, None, A=A, b=b, rcond=1e-2)
    assert "fixed scratch" in str(e.value)
    tb.free()
    # another route than the FP64 Tikhonov one is refused
    import ctypes
    from paper_2608_07017_amd._lib import WosSolveInfo
    tb2, s2, b2 = _toolbox(120, 6)
    A2, bb2, f2, g2 = _problem(s2, b2)
    f_, g_, A_, b_, c_, co = tb2._coeffs(f2, g2, "linear", A2, bb2, None, rcond=1e-2, solver="tsvd")
    u2 = torch.zeros(tb2.n, dtype=torch.float64, device="cuda")
    info = WosSolveInfo()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    st = P.lib().wos_solve_noalloc(tb2._h, ctypes.byref(co), ptr(f_), ptr(g_), ptr(u2), None, None,
                                   ctypes.byref(info), None)
    assert st == -1 and b"TIKHONOV" in P.lib().wos_last_error()
    tb2.free()
