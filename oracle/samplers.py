"""Samplers of the refined estimators (oracle).

Prop. "removing singularities" and Rem. "MC_no_singular":

* Y has the ball-Green density f_Y = -2 d G_B(0,y) of Prop. "U_0 and DU_0"
  (eq. density Green).  It is never sampled directly:
  - d = 2 (part (i.1)): R = median of three uniforms ~ Beta(2,2), Y = R Z,
    and every A/B tally is re-weighted by omega = -(2/3) ln R / (1 - R)
    (the ratio of the radial law of f_Y, -4 t ln t, to Beta(2,2), 6t(1-t));
  - d = 2, the exact law (also part (i.1)): R = exp((1 + W_{-1}(-U/e))/2)
    with the lower branch of the Lambert W function, weight 1, U the
    first of the same three uniforms (``lambert_radius``; the paper uses
    the median representation for want of a Lambert W in its framework);
  - d = 3 (part (i.2)): R = median of three uniforms ~ Beta(2,2) and
    Y = R^{1/(d-2)} Z = R Z has exactly the law f_Y (omega = 1).  The
    paper's general statement "U_(2) ~ Beta(2/(d-2), 2)" holds only for
    d = 3, which is the only d >= 3 supported here.
* The singular ball term of the gradient (part (ii)) uses S = 1 - sqrt(U)
  and Z on the sphere: E{Y~ (|Y~|^-d - 1) f(x + r Y~)} =
  (d/2) E{sum_{k<d} S^k Z f(x + r S Z)}.  With the prefactor 2 r / d of
  eq. (grad_U0_rep_intro) the ball-term weight is r * sum_{k<d} S^k * Z.
* Directions uniform on the unit sphere (eq. Uk iid): d = 2 by an angle,
  theta = 2 pi a; d = 3 by Archimedes' theorem, z = 2u - 1 uniform,
  phi = 2 pi u'.

Pinned by tests/test_oracle_samplers.py: the CDF of Beta(2,2), the law of
S (CDF 2t - t^2), E[omega] = 1 and E[omega R^2] = 1/4 (the radial moments
of f_Y), the first two moments of the sphere directions, the ball-term
identity integrated in closed form, and the Lambert radius against the
radial distribution function r^2 (1 - 2 ln r) of f_Y.
"""
import numpy as np


def median3(u1, u2, u3):
    return np.median(np.stack([u1, u2, u3]), axis=0)


def lambert_radius(u):
    """The exact radial law of Y in d = 2 (Prop. "removing singularities"
    (i.1)): R = exp((1 + W_{-1}(-U/e)) / 2), W_{-1} the lower real branch of
    the Lambert W function (scipy's lambertw, branch -1); used with weight 1."""
    from scipy.special import lambertw
    u = np.asarray(u, dtype=np.float64)
    w = lambertw(-u / np.e, -1).real
    # at the branch point y = -1/e (u = 1) W_{-1} = -1 by definition; scipy
    # returns NaN for the rounded -1/e itself
    w = np.where(np.isnan(w), -1.0, w)
    return np.exp(0.5 * (1.0 + w))


def omega(R, dim):
    """Importance weight of the d = 2 Beta(2,2) substitute for f_Y; 1 for d = 3."""
    R = np.asarray(R, dtype=np.float64)
    if dim == 2:
        return -(2.0 / 3.0) * np.log(R) / (1.0 - R)
    if dim == 3:
        return np.ones_like(R)
    raise ValueError("only d = 2 and d = 3 are supported")


def s_of_u(u):
    """S = 1 - sqrt(U): density 2(1-s) on (0,1)."""
    return 1.0 - np.sqrt(np.asarray(u, dtype=np.float64))


def ball_weight_poly(S, dim):
    """sum_{k=0}^{d-1} S^k."""
    S = np.asarray(S, dtype=np.float64)
    return sum(S ** k for k in range(dim))


def sphere(dim, us):
    """Uniform direction on the unit sphere from d-1 uniforms (list of arrays)."""
    if dim == 2:
        th = 2.0 * np.pi * np.asarray(us[0], dtype=np.float64)
        return np.stack([np.cos(th), np.sin(th)], axis=-1)
    if dim == 3:
        z = 2.0 * np.asarray(us[0], dtype=np.float64) - 1.0
        ph = 2.0 * np.pi * np.asarray(us[1], dtype=np.float64)
        s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
        return np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=-1)
    raise ValueError("only d = 2 and d = 3 are supported")
