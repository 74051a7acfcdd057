"""Pins of the oracle's samplers against the laws the paper states
(Prop. "removing singularities", Rem. "MC_no_singular")."""
import numpy as np
from scipy import stats

from oracle.philox import walk_block
import pytest

from oracle import samplers as S
from oracle.samplers import median3, omega, s_of_u, sphere, ball_weight_poly

N = 400_000


def _uniforms(block, k=4):
    return walk_block(2024, np.arange(N), 7, block)[:k]


def test_median_of_three_is_beta22():
    u = _uniforms(0)
    R = median3(u[0], u[1], u[2])
    # Beta(2,2) CDF 3t^2 - 2t^3
    ks = stats.kstest(R, lambda t: 3 * t**2 - 2 * t**3)
    assert ks.pvalue > 1e-3


def test_S_law():
    S = s_of_u(_uniforms(0)[3])
    ks = stats.kstest(S, lambda t: 2 * t - t * t)
    assert ks.pvalue > 1e-3
    assert abs(S.mean() - 1 / 3) < 6 * S.std() / np.sqrt(N)
    assert abs((S**2).mean() - 1 / 6) < 6 * (S**2).std() / np.sqrt(N)


def test_omega_reweights_beta_to_green_density():
    # Radial law of f_Y in d = 2 is -4 t ln t: E[1] = 1 and E[|Y|^2] = 1/4.
    u = _uniforms(0)
    R = median3(u[0], u[1], u[2])
    w = omega(R, 2)
    assert np.all(np.isfinite(w)) and np.all(w > 0)
    assert abs(w.mean() - 1.0) < 6 * w.std() / np.sqrt(N)
    wr = w * R * R
    assert abs(wr.mean() - 0.25) < 6 * wr.std() / np.sqrt(N)
    # d = 3: R ~ Beta(2,2) is already the radial law of f_Y, 6 t (1 - t):
    # E|Y| = 1/2, E|Y|^2 = 3/10
    assert np.all(omega(R, 3) == 1.0)
    assert abs(R.mean() - 0.5) < 6 * R.std() / np.sqrt(N)
    assert abs((R * R).mean() - 0.3) < 6 * (R * R).std() / np.sqrt(N)


def test_omega_closed_form_points():
    # -(2/3) ln R / (1 - R) at R = 1/2 is (4/3) ln 2; the limit R -> 1 is 2/3
    assert np.isclose(omega(np.array([0.5]), 2)[0], 4.0 / 3.0 * np.log(2.0))
    assert np.isclose(omega(np.array([1 - 2.0**-24]), 2)[0], 2.0 / 3.0, rtol=1e-6)


def test_sphere_moments():
    for d, blocks in ((2, [[0]]), (3, [[0, 1]])):
        u = _uniforms(1)
        Z = sphere(d, [u[i] for i in blocks[0]])
        assert np.allclose(np.linalg.norm(Z, axis=1), 1.0, atol=1e-14)
        se = 1.0 / np.sqrt(N)
        assert np.all(np.abs(Z.mean(axis=0)) < 6 * se)
        C = Z.T @ Z / N
        assert np.all(np.abs(C - np.eye(d) / d) < 6 * se)


def test_ball_term_identity_linear_f():
    # E{Y~ (|Y~|^-d - 1) Y~_1} = (d/2) E{sum_{k<d} S^k Z (S Z_1)} for Y~ uniform
    # in the unit ball.  Closed form of the left side: (1/d)(1/(2) - ... ):
    # d = 2: 1/4; d = 3: int_0^1 t^2 (t^-3 - 1) 3 t^2 dt / 3 = (1/2 - 1/5) = 3/10.
    u = _uniforms(0)
    S = s_of_u(u[3])
    ub = _uniforms(1)
    for d, lhs, Zu in ((2, 0.25, [ub[0]]), (3, 0.3, [ub[0], ub[1]])):
        Z = sphere(d, Zu)
        val = (d / 2) * ball_weight_poly(S, d) * S * Z[:, 0] * Z[:, 0]
        assert abs(val.mean() - lhs) < 6 * val.std() / np.sqrt(N)


def test_lambert_radius_has_the_green_radial_law():
    # the radial law of f_Y in d = 2 has the density -4 r ln r and the
    # distribution function F(r) = r^2 (1 - 2 ln r); R = exp((1 + W_{-1}(-u/e))/2)
    # must satisfy F(R) = u exactly (up to rounding), with R(1) = 1
    u = np.concatenate([np.linspace(1e-9, 1.0, 2001), [1e-300, 0.5]])
    R = S.lambert_radius(u)
    assert np.all((R > 0) & (R <= 1.0))
    F = R**2 * (1.0 - 2.0 * np.log(R))
    assert np.allclose(F, u, rtol=1e-11, atol=1e-15)
    assert S.lambert_radius(1.0) == pytest.approx(1.0, abs=1e-7)
