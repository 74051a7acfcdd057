"""Pins of where the oracle's walker puts each tally, entry by entry.

T7 -- every entry of A and B against the Green function of the disk and the
ball integrated over the Voronoi cell (Prop. "U_0 and DU_0", eq. density
Green, and the appendix lemma on the Green function of a ball: the binned
estimators of eqs. Estimator_A and Estimator_B have the expectations
int_{V_j} G(x_i, y) dy and int_{V_j} grad_x G(x_i, y) dy).  The quadrature
(tests/green_quadrature.py) shares nothing with the oracle; its own error is
estimated from a run at a quarter of the directions.

T8 -- U(-Lap phi / 2) = phi and grad U(-Lap phi / 2) = grad phi for
non-harmonic phi that vanish on the boundary (eq. mathcal U: U is the
inverse of -Lap/2 with zero boundary values), on all five domains.  A
harmonic source (T1, T3) cannot tell the tally point X_k + r_k Y from X_k
by the mean-value property; a non-harmonic one can.

T9 -- the harmonic extension of g = |y| on the disk and its gradient at
points of the x-axis (the paper's grad H test), against the Poisson
integral in Fourier form.

T14 -- the exit time from the unit square (its torsion function), against
the double sine series.

Each per-entry comparison allows 4.5 standard errors (per-walk, from the
same walks) plus the quadrature error plus the bias of the eps stop
(at most 2 eps / d of exit time).  tests/test_oracle_mutations.py plants
plausible mistakes in a copy of the oracle and checks that these pins fail.
"""
import numpy as np
import pytest

import workloads as W
from oracle import walker as oracle_walker
from oracle.voronoi import nearest

from green_quadrature import cell_integrals

DISK = W.unit_disk()
BALL = W.unit_ball()

T7_CASES = {
    # (domain, number of centres, walks, directions of the quadrature)
    2: (DISK, 12, 200000, 4096),
    3: (BALL, 16, 100000, 8192),
}


def per_walk_tallies(ev, centres, N, d):
    """Per-walk sums of each site's tallies by cell: A (N, m), B (d, N, m)."""
    m = len(centres)
    jv = nearest(centres, ev.ev_pts)
    jb = nearest(centres, ev.ball_pts)
    A = np.bincount(ev.ev_walk * m + jv, weights=ev.ev_tA, minlength=N * m).reshape(N, m)
    B = np.stack([np.bincount(np.arange(N) * m + jb, weights=ev.ball_w[:, a], minlength=N * m).reshape(N, m)
                  + np.bincount(ev.ev_walk * m + jv, weights=ev.ev_tB[:, a], minlength=N * m).reshape(N, m)
                  for a in range(d)])
    return A, B


def t7_zscores(walker, d, rows=(2, 7), eps=1e-5, seed=17, walks=None):
    """Largest |oracle - Green quadrature| / allowance over the entries of
    A and B of the given rows (allowance = 4.5 SE + quadrature error + the
    eps bias); <= 1 passes."""
    dom, m, N, ndir = T7_CASES[d]
    N = walks or N
    c = W.sample_sites(dom, m, 3, 0.05)
    worst = 0.0
    for i in rows:
        tb = walker.build_toolbox(dom, c, W.circle_nodes(8) if d == 2 else W.fibonacci_sphere(8), N, eps, seed,
                                  rows=[i])
        ev = walker.site_events(dom, c[i], i, np.arange(N), eps, seed)
        A, B = per_walk_tallies(ev, c, N, d)
        # the binned toolbox is the mean of the per-walk sums (same walks)
        assert np.allclose(tb["A"][0], A.mean(0), rtol=1e-10, atol=1e-14)
        assert np.allclose(tb["B"][:, 0], B.mean(1), rtol=1e-10, atol=1e-13)
        Aq, Bq = cell_integrals(c[i], c, n_dir=ndir)
        Aq4, Bq4 = cell_integrals(c[i], c, n_dir=ndir // 4)
        seA = A.std(0, ddof=1) / np.sqrt(N)
        seB = B.std(1, ddof=1) / np.sqrt(N)
        tolA = 4.5 * seA + np.abs(Aq - Aq4) / 3 + 2 * eps / d
        tolB = 4.5 * seB + np.abs(Bq - Bq4) / 3 + 2 * eps
        worst = max(worst, np.max(np.abs(tb["A"][0] - Aq) / tolA), np.max(np.abs(tb["B"][:, 0] - Bq) / tolB))
    return worst


@pytest.mark.parametrize("d", [2, 3])
def test_t7_entries_of_A_and_B_match_the_green_function(d):
    assert t7_zscores(oracle_walker, d) <= 1.0


def test_t7_quadrature_row_sums_are_the_closed_forms():
    # the quadrature itself: summed over the cells it must give E tau and its
    # gradient, (1 - |x|^2) / d and -2 x / d
    for d, (dom, m, _, ndir) in T7_CASES.items():
        c = W.sample_sites(dom, m, 3, 0.05)
        x = c[5]
        Aq, Bq = cell_integrals(x, c, n_dir=ndir // 4)
        assert np.isclose(Aq.sum(), (1 - x @ x) / d, rtol=1e-9)
        assert np.allclose(Bq.sum(1), -2 * x / d, rtol=1e-8, atol=1e-10)


# ------------------------------------------------------------------ T8
def _cube_ball_phi(x):
    """phi = prod_a x_a (1 - x_a) * (|x - c|^2 - R^2) on (0,1)^3 minus the
    ball (c = (1/2,1/2,1/2), R = 0.3): zero on both boundaries.  Returns
    phi, grad phi, -Lap phi / 2 (product rule, by hand)."""
    c = np.array([0.5, 0.5, 0.5])
    q = x * (1 - x)                        # (k, 3)
    dq = 1 - 2 * x
    u = q.prod(1)
    gu = np.stack([dq[:, a] * np.prod(np.delete(q, a, 1), 1) for a in range(3)], 1)
    lu = sum(-2 * np.prod(np.delete(q, a, 1), 1) for a in range(3))
    v = np.sum((x - c) ** 2, 1) - 0.09
    gv = 2 * (x - c)
    lv = 6.0
    phi = u * v
    grad = gu * v[:, None] + u[:, None] * gv
    lap = lu * v + 2 * np.sum(gu * gv, 1) + u * lv
    return phi, grad, -0.5 * lap


def _disk_ball_phi(d):
    # phi = (1 - |x|^4) / (2 (d + 2)), -Lap phi / 2 = |x|^2
    def f(x):
        r2 = np.sum(x * x, 1)
        return (1 - r2 * r2) / (2 * (d + 2)), -2 * r2[:, None] * x / (d + 2), r2
    return f


def _square_phi(x):
    X, Y = x[:, 0], x[:, 1]
    phi = X * (1 - X) * Y * (1 - Y)
    grad = np.stack([(1 - 2 * X) * Y * (1 - Y), X * (1 - X) * (1 - 2 * Y)], 1)
    return phi, grad, Y * (1 - Y) + X * (1 - X)


def _lshape_phi(x):
    # phi = x y (1 - x^2)(1 - y^2) vanishes on the six edges of the L-shape
    X, Y = x[:, 0], x[:, 1]
    phi = X * Y * (1 - X * X) * (1 - Y * Y)
    grad = np.stack([Y * (1 - Y * Y) * (1 - 3 * X * X), X * (1 - X * X) * (1 - 3 * Y * Y)], 1)
    return phi, grad, 3 * X * Y * (2 - X * X - Y * Y)


T8_CASES = [
    ("disk", DISK, _disk_ball_phi(2), [[0.35, -0.2], [-0.6, 0.5]]),
    ("ball", BALL, _disk_ball_phi(3), [[0.3, -0.2, 0.4]]),
    ("square", W.unit_square(), _square_phi, [[0.3, 0.6], [0.8, 0.15]]),
    ("lshape", W.l_shape(), _lshape_phi, [[-0.5, -0.4], [0.45, 0.55], [-0.3, 0.3]]),
    ("cubeball", W.cube_minus_ball(), _cube_ball_phi, [[0.15, 0.3, 0.5], [0.8, 0.85, 0.2]]),
]


def t8_zscore(walker, dom, phi_fn, pts, N=60000, eps=1e-5, seed=23):
    worst = 0.0
    for k, x in enumerate(pts):
        x = np.asarray(x, dtype=np.float64)
        phi, grad, _ = phi_fn(x[None])
        o = walker.pointwise(dom, x, 40 + k, N, eps, seed, f=lambda q: phi_fn(q)[2])
        d = len(x)
        worst = max(worst, abs(o["U"] - phi[0]) / (4.5 * o["U_se"] + 2 * eps / d),
                    np.max(np.abs(o["gradU"] - grad[0]) / (4.5 * o["gradU_se"] + 2 * eps)))
    return worst


@pytest.mark.parametrize("name,dom,phi_fn,pts", T8_CASES, ids=[c[0] for c in T8_CASES])
def test_t8_defining_functions(name, dom, phi_fn, pts):
    assert t8_zscore(oracle_walker, dom, phi_fn, pts) <= 1.0


def test_t8_sources_are_minus_half_laplacians():
    # the hand-derived -Lap phi / 2 of each case, against central differences
    rng = np.random.default_rng(0)
    h = 1e-4
    for name, dom, phi_fn, pts in T8_CASES:
        d = dom["dim"]
        x = np.asarray(pts, dtype=np.float64) + 0.01 * rng.normal(size=(len(pts), d))
        _, grad, f = phi_fn(x)
        lap = np.zeros(len(x))
        for a in range(d):
            e = np.zeros(d)
            e[a] = h
            lap += (phi_fn(x + e)[0] - 2 * phi_fn(x)[0] + phi_fn(x - e)[0]) / h ** 2
            assert np.allclose(grad[:, a], (phi_fn(x + e)[0] - phi_fn(x - e)[0]) / (2 * h), rtol=1e-6, atol=1e-9)
        assert np.allclose(f, -0.5 * lap, rtol=1e-5, atol=1e-6), name


def test_t8_defining_functions_vanish_on_the_boundary():
    from oracle.geometry import distance
    # points on each boundary (distance 0 within rounding) give phi = 0
    for name, dom, phi_fn, _ in T8_CASES:
        if dom["kind"] == "ball":
            bn = W.circle_nodes(37) if dom["dim"] == 2 else W.fibonacci_sphere(41)
        elif dom["kind"] == "box":
            bn = W.square_nodes(9)
        elif dom["kind"] == "polygon":
            bn = W.polygon_nodes(dom["verts"], 48)
        else:
            bn = np.concatenate([W.cube_face_nodes(5), W.fibonacci_sphere(30, dom["center"], dom["radius"])])
        assert np.allclose(np.abs(distance(dom, bn)), 0, atol=1e-12)
        assert np.allclose(phi_fn(bn)[0], 0, atol=1e-12), name


# ------------------------------------------------------------------ T9
def _abs_y_extension(x, terms=4000):
    """Harmonic extension of |y| (= |sin t| on the circle) and its gradient
    at points (x, 0) of the x-axis: |sin t| = 2/pi - (4/pi) sum_k cos(2kt) /
    (4k^2 - 1), so u(r, t) = 2/pi - (4/pi) sum_k r^{2k} cos(2kt) / (4k^2 - 1);
    on the axis grad u = (du/dr sign(x), 0) (du/dt = 0 there)."""
    k = np.arange(1, terms + 1)
    r = abs(x)
    u = 2 / np.pi - 4 / np.pi * np.sum(r ** (2 * k) / (4 * k * k - 1))
    du = -4 / np.pi * np.sum(2 * k * r ** (2 * k - 1) / (4 * k * k - 1))
    return u, np.array([du * np.sign(x), 0.0])


def t9_zscore(walker, N=60000, eps=1e-5, seed=29):
    worst = 0.0
    for k, x0 in enumerate([0.0, 0.3, -0.55, 0.8]):
        x = np.array([x0, 0.0])
        o = walker.pointwise(DISK, x, 60 + k, N, eps, seed, g=lambda q: np.abs(q[:, 1]))
        u, gu = _abs_y_extension(x0)
        # the terminal point is within eps of the circle, |y| is 1-Lipschitz
        worst = max(worst, abs(o["H"] - u) / (4.5 * o["H_se"] + eps),
                    np.max(np.abs(o["gradH"] - gu) / (4.5 * o["gradH_se"] + 2 * eps / max(1 - abs(x0), 0.1))))
    return worst


def test_t9_harmonic_extension_of_abs_y():
    assert t9_zscore(oracle_walker) <= 1.0


def test_t9_series_reproduces_the_boundary_data():
    # at r -> 1 on the axis the series gives |y| = 0, and at the centre the
    # mean of |sin t|, 2 / pi
    assert abs(_abs_y_extension(0.0)[0] - 2 / np.pi) < 1e-15
    assert abs(_abs_y_extension(0.999999, terms=200000)[0]) < 1e-3


# ----------------------------------------------------------------- T14
def _square_torsion(x, terms=199):
    """E tau from x in (0,1)^2: -Lap u / 2 = 1, u = 0 on the boundary:
    u = sum_{m,n odd} 32 sin(m pi x) sin(n pi y) / (pi^4 m n (m^2 + n^2))."""
    k = np.arange(1, terms + 1, 2)
    M, N = np.meshgrid(k, k, indexing="ij")
    c = 32.0 / (np.pi ** 4 * M * N * (M * M + N * N))
    sx, sy = np.sin(np.pi * k * x[0]), np.sin(np.pi * k * x[1])
    cx, cy = np.cos(np.pi * k * x[0]), np.cos(np.pi * k * x[1])
    u = np.einsum("mn,m,n->", c, sx, sy)
    g = np.array([np.einsum("mn,m,n->", c * np.pi * M, cx, sy), np.einsum("mn,m,n->", c * np.pi * N, sx, cy)])
    return u, g


def test_t14_square_torsion():
    sq = W.unit_square()
    for k, x in enumerate([[0.5, 0.5], [0.2, 0.7], [0.9, 0.4]]):
        x = np.asarray(x)
        o = oracle_walker.pointwise(sq, x, 80 + k, 60000, 1e-5, 31, f=lambda q: np.ones(len(q)))
        u, g = _square_torsion(x)
        assert abs(o["U"] - u) <= 4.5 * o["U_se"] + 1e-5
        assert np.all(np.abs(o["gradU"] - g) <= 4.5 * o["gradU_se"] + 2e-5)


def test_t14_series_solves_the_torsion_problem():
    # -Lap u / 2 = 1 by central differences (step 1e-2: O(h^2) = 1e-4), and
    # the centre value: twice the classical maximum 0.0736713 of the
    # solution of -Lap psi = 1 on the unit square
    h = 1e-2
    x = np.array([0.3, 0.6])
    lap = sum((_square_torsion(x + e)[0] - 2 * _square_torsion(x)[0] + _square_torsion(x - e)[0]) / h ** 2
              for e in (np.array([h, 0]), np.array([0, h])))
    assert abs(-0.5 * lap - 1.0) < 2e-4
    assert abs(_square_torsion(np.array([0.5, 0.5]))[0] - 2 * 0.0736713) < 2e-6
