"""p-HiSD saddle search on the GPU (wos_saddle through the C ABI) against
the oracle's p-HiSD on the exported toolbox.

Both sides run the same iteration on the same matrices.  They differ in
the summation order, in M^-1 (Newton-Schulz on the GPU, an LU solve in the
oracle; both to rounding times the condition of A) and in the rounding of
the central differences (relative eps |grad J| / h, h = 1e-6 |fbar|), so
iterates after a few steps agree to about 1e-7 relative.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import euler_lagrange as E

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


@pytest.fixture(scope="module")
def ring_tb():
    _say("GPU build disk rings 5, 1500 walks, FP64")
    tb = P.Toolbox(W.unit_disk(), _rings(5), W.circle_nodes(30), 1500, 1e-3, seed=11, precision="f64",
                   volume_samples=1 << 18)
    tb.build()
    torch.cuda.synchronize()
    mats = {k: tb.export(k).cpu().numpy().astype(np.float64) for k in ("A", "B", "H", "K", "lambda")}
    return tb, mats


def _problem(n, p, seed):
    rng = np.random.default_rng(seed)
    return 2.0 + rng.normal(size=n), 0.1 * rng.normal(size=p)


# M = I first: its call allocates no Newton-Schulz matrices, so the M = A
# call that follows on the same toolbox grows the work buffer
@pytest.mark.parametrize("precond,eta,tau", [("identity", 20.0, 20.0), ("A", 0.5, 0.5)])
def test_saddle_given_directions_matches_oracle(ring_tb, precond, eta, tau):
    tb, mats = ring_tb
    lam = mats["lambda"]
    f, g = _problem(tb.n, tb.p, 5)
    rng = np.random.default_rng(6)
    V0 = rng.normal(size=(2, tb.m))
    fb0 = 1.0 + 0.1 * rng.normal(size=tb.m)
    iters = 12
    _say("saddle precond=%s k=2 iters=%d" % (precond, iters))
    u, gu, fb, V, info = tb.saddle(f, g, 2, eta, tau, iters, fbar0=fb0, V0=V0, precond=precond)
    M = mats["A"] if precond == "A" else np.eye(tb.m)
    gr = lambda x: E.energy_grad("semilinear", mats, lam, x, g, 0.0, f)
    ref_fb, ref_V, it = E.phisd(gr, fb0, V0.T, M, eta, tau, iters)
    assert info["iters"] == it == iters
    fb, V = fb.cpu().numpy(), V.cpu().numpy()
    assert np.abs(fb - ref_fb).max() <= 1e-7 * np.abs(ref_fb).max()
    assert np.abs(V.T - ref_V).max() <= 1e-6 * np.abs(ref_V).max()
    ref_u, ref_gu = E.reconstruct(mats, ref_fb, g)
    assert np.abs(u.cpu().numpy() - ref_u).max() <= 1e-7 * np.abs(ref_u).max()
    assert info["grad_norm"] == pytest.approx(E.grad_norm(lam, gr(ref_fb)), rel=1e-5)
    assert info["grad_norm0"] == pytest.approx(E.grad_norm(lam, gr(fb0)), rel=1e-10)
    assert info["J"] == pytest.approx(E.energy_J("semilinear", mats, lam, ref_fb, g, 0.0, f), rel=1e-7)
    if precond == "A":
        assert info["ns_iters"] > 0 and info["ns_residual"] < 1e-8
        # the directions are M-orthonormal in the Gram-Schmidt sense
        G = V @ M @ V.T
        assert np.allclose(np.diag(G), 1.0, atol=1e-9) and abs(G[0, 1]) < 1e-9


def test_saddle_hessian_initialisation_matches_oracle(ring_tb):
    # the directions start as the eigenvectors of the k smallest eigenvalues
    # of the Hessian at fbar_0; fbar's update is invariant to their signs and
    # V is compared up to them.  The eigenvalue gaps are checked first.
    tb, mats = ring_tb
    lam = mats["lambda"]
    f, g = _problem(tb.n, tb.p, 7)
    fb0 = np.full(tb.m, 30.0)
    H0 = E.semilinear_hessian(mats, lam, fb0, g)
    ev, evec = np.linalg.eigh(0.5 * (H0 + H0.T))
    k = 2
    gaps = np.diff(ev[: k + 1])
    assert gaps.min() > 1e-6 * np.abs(ev).max(), "near-degenerate eigenvalues: the test needs other data"
    _say("saddle hessian init k=%d" % k)
    for iters in (1, 6):
        _, _, fb, V, info = tb.saddle(f, g, k, 0.5, 0.5, iters, fbar0=fb0, precond="A")
        gr = lambda x: E.energy_grad("semilinear", mats, lam, x, g, 0.0, f)
        ref_fb, ref_V, _ = E.phisd(gr, fb0, evec[:, :k], mats["A"], 0.5, 0.5, iters)
        fb, V = fb.cpu().numpy(), V.cpu().numpy().T
        assert np.abs(fb - ref_fb).max() <= 1e-6 * np.abs(ref_fb).max()
        sgn = np.sign(np.sum(V * ref_V, axis=0))
        assert np.abs(V * sgn - ref_V).max() <= 1e-5 * np.abs(ref_V).max()


def test_saddle_stops_at_the_tolerance(ring_tb):
    # with a tolerance that every norm meets, the run ends at the first
    # check (iteration check_every)
    tb, mats = ring_tb
    f, g = _problem(tb.n, tb.p, 9)
    _, _, _, _, info = tb.saddle(f, g, 1, 0.5, 0.5, 400, fbar0=1.0, V0=np.ones((1, tb.m)), precond="A",
                                 energy="semilinear", tol=1e30, check_every=7)
    assert info["iters"] == 7


def test_saddle_invalid_options(ring_tb):
    tb, _ = ring_tb
    f, g = np.ones(tb.n), np.zeros(tb.p)
    with pytest.raises(ValueError):
        tb.saddle(f, g, 0, 1.0, 1.0, 5)
    for kw in ({"k": 1, "eta": 0.0, "tau": 1.0, "max_iter": 5}, {"k": 1, "eta": 1.0, "tau": 0.0, "max_iter": 5},
               {"k": 1, "eta": 1.0, "tau": 1.0, "max_iter": 0},
               {"k": 1, "eta": 1.0, "tau": 1.0, "max_iter": 5, "energy": "plaplace", "p_exp": 2.0},
               {"k": 1, "eta": 1.0, "tau": 1.0, "max_iter": 5, "energy": "elliptic", "V0": np.ones((1, tb.m))}):
        with pytest.raises(P.WosError):
            tb.saddle(f, g, **kw)
    # dependent directions
    with pytest.raises(P.WosError):
        tb.saddle(f, g, 2, 1.0, 1.0, 5, V0=np.ones((2, tb.m)), precond="identity")


def test_saddle_preconditioner_needs_square_toolbox():
    dom = W.unit_disk()
    tb = P.Toolbox(dom, W.sample_sites(dom, 30, 3, 1e-3), W.circle_nodes(20), 100, 1e-3, seed=3, precision="f64",
                   volume_samples=1 << 14, vcentres=W.sample_sites(dom, 20, 4, 1e-3))
    tb.build()
    f, g = np.ones(30), np.zeros(20)
    with pytest.raises(P.WosError):
        tb.saddle(f, g, 1, 1.0, 1.0, 5, V0=np.ones((1, 20)), precond="A")
    _, _, fb, V, info = tb.saddle(f, g, 1, 1.0, 1.0, 3, V0=np.ones((1, 20)), precond="identity")
    assert info["iters"] == 3 and fb.numel() == 20
    # with M = I the batched gradients run over the rectangular A and B
    # (n = 30 sites, m = 20 cells): against the oracle, k = 2
    mats = {key: tb.export(key).cpu().numpy().astype(np.float64) for key in ("A", "B", "H", "K", "lambda")}
    lam = mats["lambda"]
    f2, g2 = _problem(30, 20, 25)
    rng = np.random.default_rng(26)
    V0 = rng.normal(size=(2, 20))
    _, _, fb, V, info = tb.saddle(f2, g2, 2, 20.0, 20.0, 6, fbar0=1.0, V0=V0, precond="identity")
    gr = lambda x: E.energy_grad("semilinear", mats, lam, x, g2, 0.0, f2)
    ref_fb, ref_V, _ = E.phisd(gr, np.ones(20), V0.T, np.eye(20), 20.0, 20.0, 6)
    assert np.abs(fb.cpu().numpy() - ref_fb).max() <= 1e-7 * np.abs(ref_fb).max()
    assert np.abs(V.cpu().numpy().T - ref_V).max() <= 1e-6 * np.abs(ref_V).max()


def test_saddle_paper_semilinear_s800_index1():
    # The paper's example Lap u + u^2 = 800 sin(pi x) sin(pi y), u = 0 on
    # the unit square, on its 20 x 20 layout (1e5 walks/site, FP64), with
    # its p-HiSD parameters (M = A, fbar_0 = 1000, eta = 20, tau = 10,
    # directions from the Hessian) and k = 1, run to its final gradient norm
    # 1e-6.  The result is a critical point whose Hessian (the oracle's, on
    # the exported toolbox) has exactly one negative eigenvalue, unlike the
    # minimum Adam reaches.
    sites, bn = W.paper_square_layout()
    _say("GPU build paper square, 1e5 walks")
    tb = P.Toolbox(W.unit_square(), sites, bn, 100000, 1e-4, seed=11, precision="f64", volume_samples=1 << 20)
    tb.build()
    torch.cuda.synchronize()
    mats = {k: tb.export(k).cpu().numpy().astype(np.float64) for k in ("A", "B", "H", "K", "lambda")}
    lam = mats["lambda"]
    f = 800.0 * np.sin(np.pi * sites[:, 0]) * np.sin(np.pi * sites[:, 1])
    g = np.zeros(tb.p)
    _say("saddle s=800 k=1")
    u, _, fb, _, info = tb.saddle(f, g, 1, 20.0, 10.0, 20000, fbar0=1000.0, precond="A", tol=1e-6, check_every=50)
    _say("  %d iters, grad norm %.2e, J %.4g, %.2f s" % (info["iters"], info["grad_norm"], info["J"], info["seconds"]))
    assert info["iters"] < 20000 and info["grad_norm"] <= 1e-6
    fb = fb.cpu().numpy()
    gr = E.energy_grad("semilinear", mats, lam, fb, g, 0.0, f)
    assert E.grad_norm(lam, gr) == pytest.approx(info["grad_norm"], rel=1e-6)
    Hf = E.semilinear_hessian(mats, lam, fb, g)
    ev = np.linalg.eigvalsh(0.5 * (Hf + Hf.T))
    assert np.sum(ev < 0) == 1
    _, _, fmin, _ = tb.minimize(f, g, 0.0, 1.0, 30000, fbar0=1.0, energy="semilinear", tol=1e-6, check_every=50)
    Hm = E.semilinear_hessian(mats, lam, fmin.cpu().numpy(), g)
    assert np.sum(np.linalg.eigvalsh(0.5 * (Hm + Hm.T)) < 0) == 0


@pytest.mark.parametrize("rings,k", [(4, 1), (4, 2), (4, 4), (5, 2)])
def test_saddle_fp32_toolbox_batched_gradients_match_oracle(rings, k):
    # FP32 toolboxes take the batched gradients (the 2k + 1 points of an
    # iteration in one pass over A and B): with m % 4 == 0 (4 rings, 48
    # sites) the 4-wide kernels, otherwise (5 rings, 75 sites) the generic
    # ones; the FP64 tests above take the generic FP64 ones.  The exported
    # FP32 entries are exact in FP64, so the oracle runs on the same
    # matrices.
    _say("GPU build disk rings %d, FP32; saddle k=%d" % (rings, k))
    tb = P.Toolbox(W.unit_disk(), _rings(rings), W.circle_nodes(24), 1500, 1e-3, seed=12, precision="f32",
                   volume_samples=1 << 18)
    tb.build()
    torch.cuda.synchronize()
    mats = {key: tb.export(key).cpu().numpy().astype(np.float64) for key in ("A", "B", "H", "K", "lambda")}
    lam = mats["lambda"]
    f, g = _problem(tb.n, tb.p, 15)
    rng = np.random.default_rng(16)
    V0 = rng.normal(size=(k, tb.m))
    fb0 = 1.0 + 0.1 * rng.normal(size=tb.m)
    u, _, fb, V, info = tb.saddle(f, g, k, 0.5, 0.5, 10, fbar0=fb0, V0=V0, precond="A")
    gr = lambda x: E.energy_grad("semilinear", mats, lam, x, g, 0.0, f)
    ref_fb, ref_V, _ = E.phisd(gr, fb0, V0.T, mats["A"], 0.5, 0.5, 10)
    fb, V = fb.cpu().numpy(), V.cpu().numpy()
    assert np.abs(fb - ref_fb).max() <= 1e-7 * np.abs(ref_fb).max()
    assert np.abs(V.T - ref_V).max() <= 1e-6 * np.abs(ref_V).max()
    assert info["grad_norm"] == pytest.approx(E.grad_norm(lam, gr(ref_fb)), rel=1e-5)


def test_saddle_paper_s800_four_distinct_solutions():
    # The paper finds at least four essentially distinct solutions of
    # Lap u + u^2 = 800 sin(pi x) sin(pi y): here Adam's minimum (Hessian
    # index 0) and p-HiSD's saddles for k = 1, 2, 3 (index k), all at the
    # paper's final norm, on an FP32 toolbox of its 20 x 20 layout (1e5
    # walks/site) with its parameters.  Solutions of different index are
    # not images of each other under the square's symmetries.
    sites, bn = W.paper_square_layout()
    _say("GPU build paper square, 1e5 walks, FP32")
    tb = P.Toolbox(W.unit_square(), sites, bn, 100000, 1e-4, seed=11, precision="f32", volume_samples=1 << 20)
    tb.build()
    torch.cuda.synchronize()
    mats = {key: tb.export(key).cpu().numpy().astype(np.float64) for key in ("A", "B", "H", "K", "lambda")}
    lam = mats["lambda"]
    f = 800.0 * np.sin(np.pi * sites[:, 0]) * np.sin(np.pi * sites[:, 1])
    g = np.zeros(tb.p)
    us = []
    _, _, fb, info = tb.minimize(f, g, 0.0, 1.0, 40000, fbar0=1.0, energy="semilinear", tol=1e-6, check_every=50)
    sols = [(0, fb.cpu().numpy(), info)]
    for k in (1, 2, 3):
        _say("saddle s=800 k=%d" % k)
        _, _, fb, _, info = tb.saddle(f, g, k, 20.0, 10.0, 40000, fbar0=1000.0, precond="A", tol=1e-6,
                                      check_every=50)
        sols.append((k, fb.cpu().numpy(), info))
    for k, fb, info in sols:
        _say("  index %d: %d iters, grad norm %.2e, J %.5g" % (k, info["iters"], info["grad_norm"], info["J"]))
        assert info["iters"] < 40000 and info["grad_norm"] <= 1e-6
        Hf = E.semilinear_hessian(mats, lam, fb, g)
        assert np.sum(np.linalg.eigvalsh(0.5 * (Hf + Hf.T)) < 0) == k
        us.append(mats["A"] @ fb)
    for a in range(4):
        for b in range(a):
            assert np.linalg.norm(us[a] - us[b]) > 0.1 * max(np.linalg.norm(us[a]), np.linalg.norm(us[b]))


@pytest.mark.parametrize("energy,p_exp", [("plaplace", 3.0), ("minimal_surface", 0.0)])
def test_saddle_other_energies_match_oracle(ring_tb, energy, p_exp):
    # the batched weights for the energies whose dF/du is constant (their c
    # term is broadcast before the transposed products): 8 iterations, k = 2,
    # M = A, against the oracle's p-HiSD
    tb, mats = ring_tb
    lam = mats["lambda"]
    f, g = _problem(tb.n, tb.p, 21)
    rng = np.random.default_rng(22)
    V0 = rng.normal(size=(2, tb.m))
    fb0 = 1.0 + 0.1 * rng.normal(size=tb.m)
    _say("saddle %s k=2" % energy)
    _, _, fb, V, info = tb.saddle(f, g, 2, 0.5, 0.5, 8, fbar0=fb0, V0=V0, precond="A", energy=energy, p_exp=p_exp)
    gr = lambda x: E.energy_grad(energy, mats, lam, x, g, p_exp, f)
    ref_fb, ref_V, _ = E.phisd(gr, fb0, V0.T, mats["A"], 0.5, 0.5, 8)
    fb, V = fb.cpu().numpy(), V.cpu().numpy()
    assert np.abs(fb - ref_fb).max() <= 1e-7 * np.abs(ref_fb).max()
    assert np.abs(V.T - ref_V).max() <= 1e-6 * np.abs(ref_V).max()
    assert info["grad_norm"] == pytest.approx(E.grad_norm(lam, gr(ref_fb)), rel=1e-5)


def test_saddle_paper_s8000_distinct_solutions():
    # Lap u + u^2 = 8000 sin(pi x) sin(pi y) on the paper's square layout
    # with its walk parameters (N = 1e7, M = 30 steps, FP32) and its table's
    # runs for the minimum and the saddles of index 1..5 (Adam alpha = 10;
    # p-HiSD M = A, fbar_0 = 1000, eta = 20, tau = 10, directions from the
    # Hessian), each to its final norm 1e-6: six essentially distinct
    # solutions (none the image of another under the square's symmetries),
    # each a critical point whose Hessian (the oracle's, on the exported
    # toolbox) has exactly k negative eigenvalues.
    from paper_2608_07017_amd import search as S
    sites, bn = W.paper_square_layout()
    _say("GPU build paper square, 1e7 walks, M = 30, FP32")
    tb = P.Toolbox(W.unit_square(), sites, bn, 10 ** 7, 0.0, seed=11, precision="f32", fixed_M=30,
                   volume_samples=1 << 22)
    tb.build()
    torch.cuda.synchronize()
    mats = {key: tb.export(key).cpu().numpy().astype(np.float64) for key in ("A", "B", "H", "K", "lambda")}
    lam = mats["lambda"]
    f = 8000.0 * np.sin(np.pi * sites[:, 0]) * np.sin(np.pi * sites[:, 1])
    g = np.zeros(tb.p)
    _, _, fb, info = tb.minimize(f, g, 0.0, 10.0, 40000, fbar0=1.0, energy="semilinear", tol=1e-6, check_every=50)
    u, _ = tb.apply(fb, g)
    runs = [{"k": 0, "fbar": fb, "u": u.cpu().numpy(), "converged": info["grad_norm"] <= 1e-6}]
    for k in (1, 2, 3, 4, 5):
        _say("saddle s=8000 k=%d" % k)
        r = S.run(tb, f, g, k, 20.0, 10.0, 1000.0, 40000, 1e-6)
        _say("  %d iters, grad norm %.2e" % (r["iters"], r["grad_norm"]))
        runs.append(r)
    for r in runs:
        assert r["converged"], r["k"]
        fb = r["fbar"].cpu().numpy()
        gr = E.energy_grad("semilinear", mats, lam, fb, g, 0.0, f)
        assert E.grad_norm(lam, gr) <= 1.1e-6
        Hf = E.semilinear_hessian(mats, lam, fb, g)
        assert np.sum(np.linalg.eigvalsh(0.5 * (Hf + Hf.T)) < 0) == r["k"]
    assert len(S.distinct(runs, S.square_symmetries(sites))) == 6
    # the symmetry test itself: a reflected copy of a solution is the same one
    perms = S.square_symmetries(sites)
    assert S.same_solution(runs[1]["u"], runs[1]["u"][perms[4]], perms, 1e-12)


@pytest.mark.parametrize("precond,eta,tau,tol,iters", [("A", 0.5, 0.5, 0.0, 300), ("identity", 20.0, 20.0, 1e-300, 230),
                                                        ("A", 0.5, 0.5, 1e-300, 130)])
def test_saddle_captured_graph_iterations_are_the_same_bits(ring_tb, precond, eta, tau, tol, iters):
    """p-HiSD with blocks of iterations replayed from one captured HIP graph
    (after a first block launch by launch; blocks of 64 without a
    tolerance, of check_every = 20 with one; the tail launch by launch)
    against the launch-by-launch loop: every iterate the same bits, so the
    end point, the directions and the statistics too; calls alternate."""
    tb, mats = ring_tb
    f, g = _problem(tb.n, tb.p, 41)
    rng = np.random.default_rng(42)
    V0 = rng.normal(size=(2, tb.m))
    fb0 = 1.0 + 0.1 * rng.normal(size=tb.m)
    outs = []
    for graph in (False, True, False, True):
        u, gu, fb, V, info = tb.saddle(f, g, 2, eta, tau, iters, fbar0=fb0, V0=V0, precond=precond, tol=tol,
                                       check_every=20 if tol > 0 else 0, graph=graph)
        torch.cuda.synchronize()
        outs.append((u.cpu(), fb.cpu(), V.cpu(), info))
    for u, fb, V, info in outs[1:]:
        assert torch.equal(u, outs[0][0]) and torch.equal(fb, outs[0][1]) and torch.equal(V, outs[0][2])
        assert info["iters"] == outs[0][3]["iters"] == iters
        assert info["J"] == outs[0][3]["J"] and info["grad_norm"] == outs[0][3]["grad_norm"]
