"""Pins of the assembly, the TSVD solve and the outer loops."""
import numpy as np

import workloads as W
from oracle import linalg as L
from oracle.walker import build_toolbox
from oracle.volume import cell_weights


def _random_tb(n=12, p=5, d=2, seed=0):
    rng = np.random.default_rng(seed)
    return {"A": rng.random((n, n)), "B": rng.normal(size=(d, n, n)), "H": rng.random((n, p)),
            "K": rng.normal(size=(d, n, p))}


def test_regrouped_sums_equal_per_cell_sums():
    n, p, d = 12, 5, 2
    tb = _random_tb(n, p, d)
    rng = np.random.default_rng(1)
    lam = rng.random(n)
    M = rng.normal(size=(n, d, d))
    Ac = M @ M.transpose(0, 2, 1) + np.eye(d)
    bc = rng.normal(size=(n, d))
    cc = rng.random(n)
    Lam, Sig = L.assemble(tb, lam, Ac, bc, cc)
    A, B, H, K = tb["A"], tb["B"], tb["H"], tb["K"]
    # literal form of the paper's definitions, one cell at a time
    Lam2 = np.zeros((n, n))
    Sig2 = np.zeros((n, p))
    Bb = np.zeros((n, n))
    Kb = np.zeros((n, p))
    Hc = np.zeros((n, p))
    for i in range(n):
        Bi, Ki = B[:, i, :], K[:, i, :]
        Lam2 += lam[i] * Bi.T @ Ac[i] @ Bi
        Sig2 += lam[i] * Bi.T @ Ac[i] @ Ki
        for j in range(n):
            Bb[i, j] = lam[i] * sum(B[a, i, j] * bc[i, a] for a in range(d))
        for j in range(p):
            Kb[i, j] = lam[i] * sum(K[a, i, j] * bc[i, a] for a in range(d))
            Hc[i, j] = lam[i] * cc[i] * H[i, j]
    Lam2 += -A.T @ Bb + A.T @ np.diag(lam * cc) @ A
    Sig2 += -A.T @ Kb + A.T @ Hc
    assert np.allclose(Lam, Lam2, rtol=1e-12, atol=1e-12)
    assert np.allclose(Sig, Sig2, rtol=1e-12, atol=1e-12)


def test_tsvd_against_numpy_pinv():
    rng = np.random.default_rng(2)
    U, _ = np.linalg.qr(rng.normal(size=(30, 30)))
    V, _ = np.linalg.qr(rng.normal(size=(30, 30)))
    s = np.logspace(0, -7, 30)
    M = U @ np.diag(s) @ V.T
    r = rng.normal(size=30)
    for rcond in (1e-3, 1e-2, 1e-9):
        assert np.allclose(L.tsvd_solve(M, r, rcond), np.linalg.pinv(M, rcond=rcond) @ r, rtol=1e-9, atol=1e-9)


def test_newton_on_quadratic_energy_is_the_linear_system():
    # F = |p|^2/2 + c u^2/2 - f u: grad J = 0 is exactly eq. linear_q with
    # A = I, b = 0, c, and the paper's f = -f.  One Newton step from any h
    # lands on it.
    tb = _random_tb(10, 4, 2, 3)
    tb["B"] *= 3
    rng = np.random.default_rng(4)
    lam = rng.random(10)
    f = rng.normal(size=10)
    g = rng.normal(size=4)
    c = rng.random(10)
    lin = L.solve_linear(tb, lam, -f, g, ccoef=c, rcond=1e-14)
    h = L.newton(tb, lam, g, dFu=lambda u: c * u - f, d2Fu=lambda u: c, rcond=1e-14, h0=rng.normal(size=10),
                 max_iter=1)["h"]
    assert np.allclose(h, lin["q"], rtol=1e-8, atol=1e-10)


def test_newton_cubic_reaches_stationary_point():
    tb = _random_tb(10, 4, 2, 5)
    rng = np.random.default_rng(6)
    lam = rng.random(10)
    f = rng.normal(size=10)
    g = rng.normal(size=4)
    out = L.newton_cubic(tb, lam, f, g, kappa=1.0, rcond=1e-14, tol=1e-12)
    assert out["grad_norm"] <= 1e-10 * out["grad_norm0"]
    # kappa = 0 is the linear problem -Lap u = f
    lin = L.solve_linear(tb, lam, -f, g, rcond=1e-14)
    out0 = L.newton_cubic(tb, lam, f, g, kappa=0.0, rcond=1e-14)
    assert np.allclose(out0["u"], lin["u"], rtol=1e-9, atol=1e-11)


def _rings(K):
    pts = []
    for k in range(1, K + 1):
        nk = 6 * k - 3
        r = (k - 0.5) / K
        th = 2 * np.pi * np.arange(nk) / nk
        pts.append(np.stack([r * np.cos(th), r * np.sin(th)], 1))
    return np.concatenate(pts)


def test_disk_poisson_end_to_end():
    # -Lap u = 1 on the unit disk, u = 0 on the boundary: u = (1 - |x|^2)/4.
    # Direct apply (1/2) A 1 and the Galerkin system both recover it, on the
    # paper's ring layout with 5 rings (75 sites).
    dom = W.unit_disk()
    sites = _rings(5)
    n = len(sites)
    bn = W.circle_nodes(30)
    tb = build_toolbox(dom, sites, bn, 1500, 1e-3, 8)
    lam, _ = cell_weights(dom, sites, 2, 1 << 18)
    exact = (1 - (sites**2).sum(1)) / 4
    u_direct, _ = L.apply_direct(tb, 0.5 * np.ones(n), np.zeros(30))
    assert np.sqrt(np.mean((u_direct - exact) ** 2)) < 0.01
    sol = L.solve_linear(tb, lam, -np.ones(n), np.zeros(30), rcond=3e-2)
    err = np.sqrt(np.sum(lam * (sol["u"] - exact) ** 2)) / np.sqrt(np.sum(lam * exact**2))
    # measured 0.049; a sign error in Lambda or in the right-hand side gives ~1
    assert err < 0.08


def test_tikhonov_matches_svd_filter_factors():
    # q = sum_j s_j / (s_j^2 + reg) v_j u_j^T r: the closed form of the
    # regularised least-squares solution from the SVD
    rng = np.random.default_rng(12)
    U, _ = np.linalg.qr(rng.normal(size=(25, 25)))
    V, _ = np.linalg.qr(rng.normal(size=(25, 25)))
    s = np.logspace(0, -6, 25)
    M = U @ np.diag(s) @ V.T
    r = rng.normal(size=25)
    q, reg = L.tikhonov_solve(M, r, 1e-2)
    assert np.isclose(reg, 1e-4 * np.max(np.sum(M * M, axis=0)))
    ref = V @ ((s / (s * s + reg)) * (U.T @ r))
    assert np.allclose(q, ref, rtol=1e-9, atol=1e-12)


def test_tikhonov_tends_to_the_inverse_for_a_well_conditioned_matrix():
    rng = np.random.default_rng(13)
    M = rng.normal(size=(12, 12)) + 6 * np.eye(12)
    r = rng.normal(size=12)
    q, _ = L.tikhonov_solve(M, r, 1e-7)
    assert np.allclose(q, np.linalg.solve(M, r), rtol=1e-9, atol=1e-11)


def test_symmetric_regularised_solve_matches_eigen_filter():
    rng = np.random.default_rng(14)
    Q, _ = np.linalg.qr(rng.normal(size=(20, 20)))
    e = np.logspace(1, -7, 20)
    M = Q @ np.diag(e) @ Q.T
    r = rng.normal(size=20)
    x, reg = L.sym_reg_solve(M, r, 1e-3)
    assert np.isclose(reg, 1e-3 * np.max(np.diag(M)))
    assert np.allclose(x, Q @ ((Q.T @ r) / (e + reg)), rtol=1e-9, atol=1e-12)


def test_regularised_newton_reaches_the_regularised_stationary_point():
    # at convergence the step vanishes: grad J(h) = 0 up to the regularised
    # solve, which for an invertible Hessian means grad J = 0
    tb = _random_tb(10, 4, 2, 5)
    tb["B"] *= 3
    rng = np.random.default_rng(6)
    lam = rng.random(10)
    f = rng.normal(size=10)
    g = rng.normal(size=4)
    res = L.newton_cubic(tb, lam, f, g, kappa=0.5, rcond=1e-12, tol=1e-12, max_iter=60, solver="tikhonov")
    assert res["grad_norm"] <= 1e-9 * res["grad_norm0"]


def _kirchhoff_inverse(w):
    """The real root u of u + u^3 / 3 = w (Cardano: u^3 + 3 u - 3 w = 0)."""
    s = np.sqrt(2.25 * w * w + 1.0)
    return np.cbrt(1.5 * w + s) + np.cbrt(1.5 * w - s)


def test_t16_picard_agrees_with_the_kirchhoff_transform():
    # -div((1 + u^2) grad u) = f becomes -Lap w = f for w = u + u^3/3
    # (grad w = (1 + u^2) grad u), with w = g + g^3/3 on the boundary: a
    # second, linear route to the same solution.  On one toolbox the Picard
    # fixed point and the transformed linear solve agree to within their
    # discretisation error against the manufactured solution, while dropping
    # the coefficient (a = 1) does not.
    dom = W.unit_disk()
    sites = _rings(5)
    n = len(sites)
    bn = W.circle_nodes(30)
    tb = build_toolbox(dom, sites, bn, 1500, 1e-3, 8)
    lam, _ = cell_weights(dom, sites, 2, 1 << 18)

    def uex(x):
        return 0.8 + 0.6 * x[:, 0] - 0.5 * x[:, 1] + 0.4 * x[:, 0] * x[:, 1]

    def grad(x):
        return np.stack([0.6 + 0.4 * x[:, 1], -0.5 + 0.4 * x[:, 0]], 1)

    # u_ex is harmonic, so f = -(1 + u^2) Lap u - 2 u |grad u|^2 = -2 u |grad u|^2
    f = -2.0 * uex(sites) * np.sum(grad(sites) ** 2, 1)
    g = uex(bn)
    pic = L.picard_quasilinear(tb, lam, f, g, rcond=3e-2, tol=1e-12)
    w = L.solve_linear(tb, lam, -f, g + g ** 3 / 3, rcond=3e-2)["u"]
    u_k = _kirchhoff_inverse(w)
    assert np.allclose(u_k + u_k ** 3 / 3, w, rtol=1e-13, atol=1e-13)
    nrm = lambda v: np.sqrt(np.sum(lam * v * v))
    ue = uex(sites)
    err_p, err_k = nrm(pic["u"] - ue), nrm(u_k - ue)
    gap = nrm(pic["u"] - u_k)
    assert err_p < 0.05 * nrm(ue) and err_k < 0.05 * nrm(ue)
    assert gap <= max(err_p, err_k)
    lin = L.solve_linear(tb, lam, -f, g, rcond=3e-2)["u"]    # the coefficient dropped
    assert nrm(lin - u_k) > 3 * max(err_p, err_k)
