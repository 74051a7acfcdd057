"""Pins of the Euler-Lagrange route: J, its gradient, Adam, and the disk's
p-torsion closed form."""
import numpy as np
import pytest

import workloads as W
from oracle import euler_lagrange as E
from oracle import linalg as L
from oracle.volume import cell_weights
from oracle.walker import build_toolbox


def _random_tb(n=10, p=4, d=2, seed=0):
    rng = np.random.default_rng(seed)
    return {"A": rng.random((n, n)), "B": rng.normal(size=(d, n, n)), "H": rng.random((n, p)),
            "K": rng.normal(size=(d, n, p))}


@pytest.mark.parametrize("P", [1.5, 2.0, 3.0, 5.0])
def test_gradient_matches_central_differences_of_J(P):
    tb = _random_tb(9, 4, 2, 1)
    rng = np.random.default_rng(2)
    lam = rng.random(9)
    f = rng.normal(size=9)
    g = rng.normal(size=4)
    fb = rng.normal(size=9)
    gr = E.plaplace_grad(tb, lam, fb, g, P, f)
    h = 1e-6
    fd = np.array([(E.plaplace_J(tb, lam, fb + h * e, g, P, f) - E.plaplace_J(tb, lam, fb - h * e, g, P, f)) / (2 * h)
                   for e in np.eye(9)])
    assert np.allclose(gr, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def test_quadratic_energy_gradient_is_the_linear_residual():
    # P = 2: F = |p|^2/2 - f u, so grad J = Lambda0 fbar + Sigma0 g - A^T (lam f)
    # with Lambda0 = sum_i lam_i B_i^T B_i (the regrouped sums of the linear
    # route, coded separately)
    tb = _random_tb(10, 4, 2, 3)
    rng = np.random.default_rng(4)
    lam, f, g, fb = rng.random(10), rng.normal(size=10), rng.normal(size=4), rng.normal(size=10)
    L0, S0 = L._grad_pairs(tb["B"], tb["K"], lam, None)
    ref = L0 @ fb + S0 @ g - tb["A"].T @ (lam * f)
    assert np.allclose(E.plaplace_grad(tb, lam, fb, g, 2.0, f), ref, rtol=1e-12, atol=1e-12)


def test_adam_first_step_has_length_alpha():
    # m1 = (1-b1) g, v1 = (1-b2) g^2, alpha_1 = alpha sqrt(1-b2)/(1-b1):
    # the first step is alpha g / (|g| + eps / sqrt(1 - b2)) = alpha sign(g)
    g0 = np.array([3.0, -0.5, 1e-3, -20.0])
    f1, it = E.adam(lambda x: g0, np.zeros(4), 0.01, 1)
    assert it == 1
    assert np.allclose(f1, -0.01 * g0 / (np.abs(g0) + 1e-10 / np.sqrt(1 - 0.999)), rtol=1e-12, atol=0)
    assert np.allclose(np.abs(f1), 0.01, rtol=1e-5)


def test_adam_minimises_a_separable_quadratic():
    c = np.array([1.0, 10.0, 0.1, 3.0])
    t = np.array([0.5, -1.0, 2.0, 0.0])
    f, it = E.adam(lambda x: c * (x - t), np.ones(4), 0.01, 20000)
    assert np.allclose(f, t, atol=2e-3)


def test_adam_route_at_P2_reaches_the_linear_solution():
    # the two routes of the paper coincide for the quadratic energy: the
    # minimiser of J solves Lambda0 fbar = A^T (lam f) - Sigma0 g
    tb = _random_tb(8, 3, 2, 5)
    rng = np.random.default_rng(6)
    lam = 0.5 + rng.random(8)
    f, g = rng.normal(size=8), rng.normal(size=3)
    L0, S0 = L._grad_pairs(tb["B"], tb["K"], lam, None)
    ref = np.linalg.solve(L0, tb["A"].T @ (lam * f) - S0 @ g)
    out = E.minimize_plaplace(tb, lam, f, g, 2.0, alpha=0.01, max_iter=40000, f0=0.0)
    assert np.allclose(out["fbar"], ref, atol=5e-3 * np.abs(ref).max())
    assert out["grad_norm"] < 1e-3


def test_adam_stops_at_the_tolerance():
    tb = _random_tb(8, 3, 2, 7)
    rng = np.random.default_rng(8)
    lam = 0.5 + rng.random(8)
    f, g = rng.normal(size=8), rng.normal(size=3)
    out = E.minimize_plaplace(tb, lam, f, g, 2.0, alpha=0.01, max_iter=40000, f0=0.0, tol=1e-2, check_every=10)
    assert out["iters"] < 40000 and out["iters"] % 10 == 0
    assert out["grad_norm"] <= 1e-2


@pytest.mark.parametrize("P", [1.5, 2.0, 3.0, 5.0, 10.0])
def test_torsion_closed_form_solves_the_radial_p_laplace_equation(P):
    # -Lap_p u = (1/r) d/dr (r |u'|^(P-2) u') = -1 for radial u, u(1) = 0;
    # checked by central differences at interior radii
    assert E.plaplace_torsion_disk(np.array([[1.0, 0.0]]), P)[0] == pytest.approx(0.0, abs=1e-15)
    h = 1e-4

    def u(r):
        return E.plaplace_torsion_disk(np.stack([r, np.zeros_like(r)], -1), P)

    def flux(r):
        du = (u(r + h) - u(r - h)) / (2 * h)
        return r * np.abs(du) ** (P - 2) * du

    for r in (0.3, 0.5, 0.8):
        r = np.array([r])
        lap = (flux(r + h) - flux(r - h)) / (2 * h) / r
        assert lap[0] == pytest.approx(-1.0, rel=1e-4)
    x = np.random.default_rng(0).uniform(-0.7, 0.7, size=(5, 2))
    if P == 2.0:
        assert np.allclose(E.plaplace_torsion_disk(x, 2.0), (1 - (x**2).sum(1)) / 4, rtol=1e-14)


def test_disk_torsion_end_to_end_early_stopped():
    # The route on an oracle toolbox (the paper's ring layout, 5 rings,
    # 1500 walks) with the paper's Adam parameters (fbar_0 = 1,
    # alpha = 1e-3) reaches the p-torsion function after 2000 iterations
    # (measured relative errors 0.055 at P = 2, 0.084 at P = 1.5).  Run on,
    # Adam drifts to the exact minimiser of this Monte Carlo J, whose error
    # is larger (0.66 at P = 2: the unregularised discrete problem with as
    # many unknowns as cells is ill-posed in its oscillating directions).
    dom = W.unit_disk()
    K = 5
    pts = []
    for k in range(1, K + 1):
        nk = 6 * k - 3
        th = 2 * np.pi * np.arange(nk) / nk
        pts.append(np.stack([(k - 0.5) / K * np.cos(th), (k - 0.5) / K * np.sin(th)], 1))
    sites = np.concatenate(pts)
    n = len(sites)
    bn = W.circle_nodes(30)
    tb = build_toolbox(dom, sites, bn, 1500, 1e-3, 8)
    lam, _ = cell_weights(dom, sites, 2, 1 << 18)
    for P, bound in ((2.0, 0.1), (1.5, 0.15)):
        exact = E.plaplace_torsion_disk(sites, P)
        out = E.minimize_plaplace(tb, lam, np.ones(n), np.zeros(30), P, alpha=1e-3, max_iter=2000, f0=1.0)
        err = np.sqrt(np.sum(lam * (out["u"] - exact) ** 2)) / np.sqrt(np.sum(lam * exact**2))
        assert err < bound


def test_interpolation_reproduces_affine_fields():
    # u(x) = a.x + b with its exact gradient at the sites: the
    # gradient-enhanced form is exact everywhere, whatever the cells
    rng = np.random.default_rng(9)
    for d in (2, 3):
        sites = rng.uniform(-1, 1, size=(50, d))
        a, b = rng.normal(size=d), 0.7
        u = sites @ a + b
        gu = np.tile(a[:, None], (1, 50))
        x = rng.uniform(-1, 1, size=(400, d))
        v, i = E.interpolate(sites, u, gu, x)
        assert np.allclose(v, x @ a + b, rtol=0, atol=1e-13)
        # without the gradient: the value of the nearest site (brute force)
        v0, i0 = E.interpolate(sites, u, None, x)
        d2 = ((x[:, None, :] - sites[None, :, :]) ** 2).sum(2)
        assert np.array_equal(i0, np.argmin(d2, axis=1)) and np.array_equal(v0, u[i0])
        # at the sites themselves: u_i
        vs, isite = E.interpolate(sites, u, gu, sites)
        assert np.array_equal(isite, np.arange(50)) and np.allclose(vs, u, rtol=0, atol=1e-14)


@pytest.mark.parametrize("energy", ["minimal_surface", "semilinear"])
def test_other_energies_gradient_matches_central_differences(energy):
    tb = _random_tb(9, 4, 2, 21)
    tb["A"] *= 0.3  # keeps u moderate for the cubic
    rng = np.random.default_rng(22)
    lam, f, g, fb = rng.random(9), rng.normal(size=9), rng.normal(size=4), 0.5 * rng.normal(size=9)
    gr = E.energy_grad(energy, tb, lam, fb, g, 0.0, f)
    h = 1e-6
    fd = np.array([(E.energy_J(energy, tb, lam, fb + h * e, g, 0.0, f)
                    - E.energy_J(energy, tb, lam, fb - h * e, g, 0.0, f)) / (2 * h) for e in np.eye(9)])
    assert np.allclose(gr, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def test_semilinear_gradient_is_the_regrouped_residual():
    # F = |p|^2/2 - u^3/3 + f u: grad J = Lambda0 fbar + Sigma0 g + A^T (lam (f - u^2))
    tb = _random_tb(10, 4, 2, 23)
    rng = np.random.default_rng(24)
    lam, f, g, fb = rng.random(10), rng.normal(size=10), rng.normal(size=4), rng.normal(size=10)
    L0, S0 = L._grad_pairs(tb["B"], tb["K"], lam, None)
    u = tb["A"] @ fb + tb["H"] @ g
    ref = L0 @ fb + S0 @ g + tb["A"].T @ (lam * (f - u * u))
    assert np.allclose(E.energy_grad("semilinear", tb, lam, fb, g, 0.0, f), ref, rtol=1e-12, atol=1e-12)


def test_minimal_surface_of_small_slope_is_the_quadratic_energy():
    # sqrt(1 + |p|^2) = 1 + |p|^2/2 + O(|p|^4): for tiny data the gradients
    # of the two energies agree to the fourth order
    tb = _random_tb(8, 3, 2, 25)
    rng = np.random.default_rng(26)
    lam, g, fb = rng.random(8), 1e-4 * rng.normal(size=3), 1e-4 * rng.normal(size=8)
    f = np.zeros(8)
    a = E.energy_grad("minimal_surface", tb, lam, fb, g, 0.0, f)
    b = E.energy_grad("plaplace", tb, lam, fb, g, 2.0, f)
    _, gu = L.reconstruct(tb, fb, g)
    s = float(np.max(np.sum(gu * gu, axis=0)))  # the gap is O(|p|^2) relative
    assert s < 1e-5
    assert np.allclose(a, b, rtol=0, atol=s * np.abs(b).max() * 8)
    assert not np.allclose(a, b, rtol=0, atol=1e-3 * s * np.abs(b).max())  # but not zero


def _saddle_quadratic(m, negs, seed):
    # J = 1/2 x^T H x - b^T x with H = Q diag(e) Q^T, `negs` negative
    # eigenvalues: the unique critical point is H^-1 b, a saddle of index negs
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(m, m)))
    e = np.concatenate([-(1.0 + np.arange(negs)), 1.0 + rng.random(m - negs) * 3])
    H = (Q * e) @ Q.T
    b = rng.normal(size=m)
    return H, b, Q, e


@pytest.mark.parametrize("k", [1, 2])
def test_phisd_finds_the_saddle_of_a_quadratic_and_its_unstable_space(k):
    # M = I: the fixed point is the critical point H^-1 b, and V spans the
    # eigenvectors of the k negative eigenvalues (the unstable directions)
    H, b, Q, e = _saddle_quadratic(8, k, 31)
    rng = np.random.default_rng(32)
    V0 = Q[:, :k] + 0.3 * rng.normal(size=(8, k))
    f, V, it = E.phisd(lambda x: H @ x - b, rng.normal(size=8), V0, np.eye(8), 0.1, 0.1, 3000)
    assert np.allclose(f, np.linalg.solve(H, b), atol=1e-8)
    proj = Q[:, :k] @ (Q[:, :k].T @ V)  # V lies in span(Q[:, :k])
    assert np.allclose(proj, V, atol=1e-6)
    assert np.allclose(V.T @ V, np.eye(k), atol=1e-10)


def test_phisd_with_a_preconditioner_reaches_the_same_saddle():
    # an SPD M changes the path, not the critical point; the directions are
    # M-orthonormal at every step
    H, b, Q, e = _saddle_quadratic(8, 1, 33)
    rng = np.random.default_rng(34)
    G = rng.normal(size=(8, 8))
    M = G @ G.T / 8 + np.eye(8)
    f, V, it = E.phisd(lambda x: H @ x - b, np.zeros(8), Q[:, :1] + 0.2 * rng.normal(size=(8, 1)), M, 0.05, 0.05,
                       4000)
    assert np.allclose(f, np.linalg.solve(H, b), atol=1e-8)
    assert np.allclose(V.T @ M @ V, np.eye(1), atol=1e-10)


def test_phisd_stops_at_the_tolerance():
    H, b, Q, e = _saddle_quadratic(6, 1, 35)
    f, V, it = E.phisd(lambda x: H @ x - b, np.zeros(6), Q[:, :1] + 0.1, np.eye(6), 0.1, 0.1, 5000, tol=1e-6,
                       norm_fn=np.linalg.norm, check_every=10)
    assert it < 5000 and it % 10 == 0 and np.linalg.norm(H @ f - b) <= 1e-6


def test_m_orthonormalize_nonsymmetric_form():
    # x^T M y with M not symmetric: v_l^T M v_i = 0 for l < i and 1 for l = i
    rng = np.random.default_rng(36)
    M = np.eye(7) + 0.2 * rng.normal(size=(7, 7))
    M = M @ M.T + 0.3 * (rng.normal(size=(7, 7)) - rng.normal(size=(7, 7)))
    V = E.m_orthonormalize(rng.normal(size=(7, 3)), M)
    G = V.T @ M @ V
    assert np.allclose(np.diag(G), 1.0, atol=1e-12)
    assert np.allclose(np.triu(G, 1), 0.0, atol=1e-12)
    # M = I: the QR factor (up to column signs)
    X = rng.normal(size=(7, 3))
    Qr, _ = np.linalg.qr(X)
    assert np.allclose(np.abs(E.m_orthonormalize(X, np.eye(7))), np.abs(Qr), atol=1e-12)


def test_semilinear_hessian_matches_differences_of_the_gradient():
    tb = _random_tb(9, 4, 2, 37)
    tb["A"] *= 0.3
    rng = np.random.default_rng(38)
    lam, f, g, fb = rng.random(9), rng.normal(size=9), rng.normal(size=4), rng.normal(size=9)
    H = E.semilinear_hessian(tb, lam, fb, g)
    h = 1e-5
    fd = np.stack([(E.energy_grad("semilinear", tb, lam, fb + h * e, g, 0, f)
                    - E.energy_grad("semilinear", tb, lam, fb - h * e, g, 0, f)) / (2 * h) for e in np.eye(9)], 1)
    assert np.allclose(H, fd, rtol=1e-7, atol=1e-8 * np.abs(H).max())
    assert np.allclose(H, H.T, atol=1e-12 * np.abs(H).max())


def _elliptic_coef(n, d, seed):
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(n, d, d))
    return {"A": np.einsum("nab,ncb->nac", G, G) + np.eye(d), "c": rng.random(n), "w": 0.5 + rng.random(n)}


def test_elliptic_gradient_matches_central_differences():
    tb = _random_tb(9, 4, 2, 41)
    rng = np.random.default_rng(42)
    lam, f, g, fb = rng.random(9), rng.normal(size=9), rng.normal(size=4), rng.normal(size=9)
    co = _elliptic_coef(9, 2, 43)
    gr = E.energy_grad("elliptic", tb, lam, fb, g, 0.0, f, co)
    h = 1e-6
    fd = np.array([(E.energy_J("elliptic", tb, lam, fb + h * e, g, 0.0, f, co)
                    - E.energy_J("elliptic", tb, lam, fb - h * e, g, 0.0, f, co)) / (2 * h) for e in np.eye(9)])
    assert np.allclose(gr, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def test_elliptic_gradient_is_the_linear_system_with_weighted_coefficients():
    # the energy is quadratic: grad J = Lambda fbar + Sigma g - A^T (lam w f)
    # with the linear route's Lambda, Sigma for the coefficients (w A, b = 0,
    # w c) (eq. linear_q, assembled by the oracle's linear algebra)
    tb = _random_tb(10, 4, 2, 44)
    rng = np.random.default_rng(45)
    lam, f, g, fb = rng.random(10), rng.normal(size=10), rng.normal(size=4), rng.normal(size=10)
    co = _elliptic_coef(10, 2, 46)
    Lm, Sg = L.assemble(tb, lam, co["w"][:, None, None] * co["A"], None, co["w"] * co["c"])
    ref = Lm @ fb + Sg @ g - tb["A"].T @ (lam * co["w"] * f)
    assert np.allclose(E.energy_grad("elliptic", tb, lam, fb, g, 0.0, f, co), ref, rtol=1e-12, atol=1e-12)
    # and with no coefficients it is the Dirichlet energy with source: the
    # P = 2 p-Laplace gradient
    assert np.allclose(E.energy_grad("elliptic", tb, lam, fb, g, 0.0, f),
                       E.energy_grad("plaplace", tb, lam, fb, g, 2.0, f), rtol=1e-12, atol=1e-12)


def test_elliptic_example_solution_satisfies_its_equation():
    # the manufactured data of the example: f = -div(A grad u) + (A grad phi).grad u
    # + c u checked by central differences of the flux A grad u
    x = np.array([[0.3, -0.2], [-0.5, 0.4], [0.1, 0.7]])
    u, gu, f = W.elliptic_divmin_disk(x)
    h = 1e-4

    def flux(y):
        _, gy, _ = W.elliptic_divmin_disk(y)
        Ay = np.stack([[np.ones(len(y)), y[:, 0] * y[:, 1]], [y[:, 0] * y[:, 1], np.ones(len(y))]]).transpose(2, 0, 1)
        return np.einsum("nab,nb->na", Ay, gy)

    div = sum((flux(x + h * e)[:, a] - flux(x - h * e)[:, a]) / (2 * h) for a, e in enumerate(np.eye(2)))
    Agphi = np.stack([x[:, 0] + x[:, 0] * x[:, 1] ** 2, x[:, 0] ** 2 * x[:, 1] + x[:, 1]], 1)
    assert np.allclose(-div + np.sum(Agphi * gu, 1) + u, f, rtol=1e-6, atol=1e-7)
    # u vanishes on the circle; gradient by differences
    th = np.linspace(0, 2 * np.pi, 7)
    assert np.allclose(W.elliptic_divmin_disk(np.stack([np.cos(th), np.sin(th)], 1))[0], 0.0, atol=1e-15)
    gfd = np.stack([(W.elliptic_divmin_disk(x + h * e)[0] - W.elliptic_divmin_disk(x - h * e)[0]) / (2 * h)
                    for e in np.eye(2)], 1)
    assert np.allclose(gu, gfd, rtol=1e-7, atol=2e-7)  # O(h^2) truncation of the differences


def test_elliptic_div_example_solution_satisfies_its_equation():
    # the manufactured data of the example "elliptic div": f = div(A grad u)
    # + b.grad u - c u checked by central differences of the flux A grad u
    x = np.array([[0.3, -0.2], [-0.5, 0.4], [0.1, 0.7], [0.0, 0.0]])
    u, gu, f = W.elliptic_div_disk(x)
    A, b, c = W.elliptic_div_coef(x)
    h = 1e-4

    def flux(y):
        Ay, _, _ = W.elliptic_div_coef(y)
        return np.einsum("nab,nb->na", Ay, W.elliptic_div_disk(y)[1])

    div = sum((flux(x + h * e)[:, a] - flux(x - h * e)[:, a]) / (2 * h) for a, e in enumerate(np.eye(2)))
    assert np.allclose(div + np.sum(b * gu, 1) - c * u, f, rtol=1e-6, atol=1e-6)
    th = np.linspace(0, 2 * np.pi, 7)
    assert np.allclose(W.elliptic_div_disk(np.stack([np.cos(th), np.sin(th)], 1))[0], 0.0, atol=1e-15)
    gfd = np.stack([(W.elliptic_div_disk(x + h * e)[0] - W.elliptic_div_disk(x - h * e)[0]) / (2 * h)
                    for e in np.eye(2)], 1)
    assert np.allclose(gu, gfd, rtol=1e-6, atol=1e-7)
    assert np.all(np.linalg.eigvalsh(A) > 0)        # uniformly elliptic on the disk


def test_t11_discretisation_floors_of_the_disk_examples():
    # the L^2 distance between the exact solution and its piecewise-constant
    # values at the sites of the disk layout (Voronoi cells): the paper notes
    # about 8.5e-2 for "elliptic div" and about 3.1e-2 for "elliptic div min"
    # (two printed digits; Monte Carlo over 2^21 points here, whose own
    # relative error is a few 1e-4)
    sites, _ = W.paper_disk_layout()
    dom = W.unit_disk()
    for fn, paper, tol in [(W.elliptic_div_disk, 8.5e-2, 0.01), (W.elliptic_divmin_disk, 3.1e-2, 0.05)]:
        u = lambda q: fn(q)[0]
        e = W.voronoi_l2_error(dom, sites, u(sites), u, npoints=1 << 21)
        assert abs(e - paper) <= tol * paper, (fn.__name__, e)
    # the measure itself: a constant field against its own values is zero,
    # and against zero values it is |u| in L^2: |1|_L2(disk) = sqrt(pi)
    one = lambda q: np.ones(len(q))
    assert W.voronoi_l2_error(dom, sites, np.ones(len(sites)), one, npoints=1 << 16) == 0.0
    assert abs(W.voronoi_l2_error(dom, sites, np.zeros(len(sites)), one, npoints=1 << 20) - np.sqrt(np.pi)) < 5e-3
