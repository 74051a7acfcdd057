"""Pins of the oracle's toolbox estimators against closed forms.

Closed forms used (unit disk / ball, standard Brownian motion, generator
Lap/2, so U = (-Lap/2)^{-1}):
  U 1 = E tau = (1 - |x|^2)/d,                 grad U 1 = -2 x / d
  U[x_1] = x_1 (1 - |x|^2)/(d + 2),            grad U[x_1] = ((1-|x|^2) e_1 - 2 x_1 x)/(d+2)
  H g = g, grad H g = grad g for harmonic g;   H of an arc = harmonic measure
The eps-shell stop biases U 1 by at most 2 eps / d (the expected exit time
left from a point within eps of the unit sphere is below 2 eps / d).
"""
import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle.walker import build_toolbox, pointwise, site_events, bin_site

DISK = W.unit_disk()
BALL = W.unit_ball()


def _close(est, se, exact, extra=0.0, k=4.0):
    return np.all(np.abs(np.asarray(est) - np.asarray(exact)) <= k * np.asarray(se) + extra)


@pytest.mark.parametrize("dom,x,eps", [(DISK, [0.3, -0.5], 1e-3), (DISK, [0.0, 0.0], 1e-4),
                                       (BALL, [0.2, 0.1, -0.6], 1e-4)])
def test_exit_time_and_gradient(dom, x, eps):
    d = dom["dim"]
    x = np.array(x)
    o = pointwise(dom, x, 3, 60000, eps, 11, f=lambda p: np.ones(len(p)))
    exact = (1 - x @ x) / d
    assert _close(o["U"], o["U_se"], exact - eps / d, eps / d)
    assert _close(o["gradU"], o["gradU_se"], -2 * x / d, 2 * eps)


@pytest.mark.parametrize("dom,x", [(DISK, [0.45, 0.3]), (BALL, [0.3, -0.2, 0.4])])
def test_linear_source_exercises_ball_term(dom, x):
    d = dom["dim"]
    x = np.array(x)
    o = pointwise(dom, x, 5, 80000, 1e-4, 12, f=lambda p: p[:, 0])
    q = 1 - x @ x
    e1 = np.eye(d)[0]
    assert _close(o["U"], o["U_se"], x[0] * q / (d + 2), 1e-4)
    assert _close(o["gradU"], o["gradU_se"], (q * e1 - 2 * x[0] * x) / (d + 2), 1e-4)


def test_harmonic_extension_and_gradient():
    x = np.array([0.3, 0.2])
    o = pointwise(DISK, x, 1, 60000, 1e-4, 13, g=lambda p: p[:, 0] ** 2 - p[:, 1] ** 2)
    assert _close(o["H"], o["H_se"], 0.05, 2e-4)
    assert _close(o["gradH"], o["gradH_se"], [0.6, -0.4], 2e-3)
    x3 = np.array([0.1, -0.4, 0.3])
    o = pointwise(BALL, x3, 1, 60000, 1e-4, 13, g=lambda p: p[:, 0] * p[:, 2])
    assert _close(o["H"], o["H_se"], 0.03, 2e-4)
    assert _close(o["gradH"], o["gradH_se"], [0.3, 0.0, 0.1], 2e-3)


def _arc_measure(x, a, b):
    rho = np.linalg.norm(x)
    phi = np.arctan2(x[1], x[0])
    P = lambda t: (1 - rho**2) / (2 * np.pi * (1 - 2 * rho * np.cos(t - phi) + rho**2))
    return integrate.quad(P, a, b, epsabs=1e-13, limit=200)[0]


def test_H_entries_are_harmonic_measure_of_arcs():
    p = 16
    bn = W.circle_nodes(p)
    sites = np.array([[0.2, 0.5], [-0.6, 0.1]])
    N = 40000
    tb = build_toolbox(DISK, sites, bn, N, 1e-4, 21)
    for r in range(2):
        exact = np.array([_arc_measure(sites[r], 2 * np.pi * (j - 0.5) / p, 2 * np.pi * (j + 0.5) / p)
                          for j in range(p)])
        H = tb["H"][r]
        se = np.sqrt(exact * (1 - exact) / N)
        assert np.all(np.abs(H - exact) <= 4.5 * se + 1e-4)
        assert tb["Hcount"][r].sum() == N           # each walk lands in exactly one cell


def test_binned_rows_equal_pointwise_on_piecewise_constant_data():
    rng = np.random.default_rng(5)
    sites = W.sample_sites(DISK, 40, 9, 1e-3)
    bn = W.circle_nodes(24)
    phi = rng.normal(size=40)
    psi = rng.normal(size=24)
    from oracle.voronoi import nearest
    tb = build_toolbox(DISK, sites, bn, 3000, 1e-3, 31, rows=[4, 17])
    for r, i in enumerate([4, 17]):
        o = pointwise(DISK, sites[i], i, 3000, 1e-3, 31,
                      f=lambda q: phi[nearest(sites, q)], g=lambda q: psi[nearest(bn, q)])
        assert np.isclose(tb["A"][r] @ phi, o["U"], rtol=1e-12, atol=1e-14)
        assert np.allclose(tb["B"][:, r] @ phi, o["gradU"], rtol=1e-12, atol=1e-13)
        assert np.isclose(tb["H"][r] @ psi, o["H"], rtol=1e-12, atol=1e-14)
        assert np.allclose(tb["K"][:, r] @ psi, o["gradH"], rtol=1e-12, atol=1e-13)
        # row sums: A 1 is the exit-time estimate, H 1 = 1 exactly
        assert np.isclose(tb["A"][r].sum(), pointwise(DISK, sites[i], i, 3000, 1e-3, 31,
                                                      f=lambda q: np.ones(len(q)))["U"], rtol=1e-12)
        assert tb["Hcount"][r].sum() == 3000


def test_fixed_M_mode_counts_M_plus_one_tallies():
    ev = site_events(DISK, np.array([0.1, 0.2]), 0, np.arange(500), 0.0, 3, fixed_M=30)
    assert np.all(ev.nsteps == 31)
    assert len(ev.ev_tA) == 500 * 31


def test_step_cap():
    ev = site_events(DISK, np.array([0.3, 0.1]), 0, np.arange(400), 1e-12, 3, max_steps=5)
    assert ev.nsteps.max() <= 6
    assert ev.capped.sum() > 0


def test_walk_length_statistics_disk():
    # Not a pin of a closed form: guards the stopping rule (mean number of
    # steps grows like log(1/eps) on the disk).
    ev1 = site_events(DISK, np.array([0.3, 0.1]), 0, np.arange(20000), 1e-2, 3)
    ev2 = site_events(DISK, np.array([0.3, 0.1]), 0, np.arange(20000), 1e-4, 3)
    assert 2.0 < ev2.nsteps.mean() - ev1.nsteps.mean() < 8.0


def test_separate_v_partition_moves_only_the_columns():
    # Binning the same walks to another V partition (W != V) changes which
    # column a tally lands in, never the tally: row sums of A and B (and H, K,
    # which are binned to the boundary cells) are those of the W = V build,
    # and permuting the V centres permutes the columns exactly.
    import workloads as W
    dom = W.unit_disk()
    sites = W.sample_sites(dom, 6, 21, 1e-3)
    bn = W.circle_nodes(9)
    vc = W.sample_sites(dom, 11, 22, 1e-3)
    same = build_toolbox(dom, sites, bn, 150, 1e-3, 5)
    wv = build_toolbox(dom, sites, bn, 150, 1e-3, 5, vcentres=vc)
    assert wv["A"].shape == (6, 11) and wv["B"].shape == (2, 6, 11)
    assert np.allclose(wv["A"].sum(1), same["A"].sum(1), rtol=1e-12)
    assert np.allclose(wv["B"].sum(2), same["B"].sum(2), rtol=1e-12, atol=1e-14)
    assert np.array_equal(wv["Hcount"], same["Hcount"]) and np.array_equal(wv["K"], same["K"])
    perm = np.random.default_rng(3).permutation(11)
    wp = build_toolbox(dom, sites, bn, 150, 1e-3, 5, vcentres=vc[perm])
    assert np.array_equal(wp["A"], wv["A"][:, perm]) and np.array_equal(wp["B"], wv["B"][:, :, perm])


@pytest.mark.parametrize("x", [[0.3, -0.5], [0.0, 0.0]])
def test_exact_radius_sampler_closed_forms(x):
    # the exact radial law (weight 1) gives the same estimators: exit time,
    # its gradient, and the linear source on the disk
    x = np.array(x)
    o = pointwise(DISK, x, 3, 60000, 1e-4, 11, f=lambda p: np.ones(len(p)), sampler="lambert")
    assert _close(o["U"], o["U_se"], (1 - x @ x) / 2 - 1e-4 / 2, 1e-4 / 2)
    assert _close(o["gradU"], o["gradU_se"], -x, 2e-4)
    o = pointwise(DISK, x, 5, 80000, 1e-4, 12, f=lambda p: p[:, 0], sampler="lambert")
    q = 1 - x @ x
    assert _close(o["U"], o["U_se"], x[0] * q / 4, 1e-4)
    assert _close(o["gradU"], o["gradU_se"], (q * np.eye(2)[0] - 2 * x[0] * x) / 4, 1e-4)


def test_site_functionals_means_and_invariants():
    # The per-walk functionals behind the per-site moments: their means are
    # the binned rows applied to phi / psi (a different route: one bincount
    # per walk, not per cell), the variance of c_H vanishes for psi = 1, and
    # |c_K|^2 = |w|^2 = (d / r0)^2 on every walk for psi = 1 (w = d/r0 U_1
    # with U_1 on the unit sphere).
    from oracle.walker import site_functionals
    rng = np.random.default_rng(8)
    for dom, n, p in [(DISK, 30, 20), (BALL, 24, 18)]:
        d = dom["dim"]
        sites = W.sample_sites(dom, n, 4, 1e-3)
        bn = W.circle_nodes(p) if d == 2 else W.fibonacci_sphere(p)
        phi = rng.normal(size=n)
        psi = rng.normal(size=p)
        i = 7
        tb = build_toolbox(dom, sites, bn, 2000, 1e-3, 17, rows=[i])
        cA, cB, cH, cK = site_functionals(dom, sites[i], i, 2000, 1e-3, 17, sites, bn, phi, psi)
        assert np.isclose(cA.mean(), tb["A"][0] @ phi, rtol=1e-12, atol=1e-14)
        assert np.allclose(cB.mean(0), tb["B"][:, 0] @ phi, rtol=1e-12, atol=1e-13)
        assert np.isclose(cH.mean(), tb["H"][0] @ psi, rtol=1e-12, atol=1e-14)
        assert np.allclose(cK.mean(0), tb["K"][:, 0] @ psi, rtol=1e-12, atol=1e-13)
        ones_v, ones_b = np.ones(n), np.ones(p)
        _, _, cH1, cK1 = site_functionals(dom, sites[i], i, 2000, 1e-3, 17, sites, bn, ones_v, ones_b)
        assert np.all(cH1 == 1.0)
        r0 = float(np.min(np.abs(1.0 - np.linalg.norm(sites[i]))))
        assert np.allclose((cK1 ** 2).sum(1), (d / r0) ** 2, rtol=1e-12)
