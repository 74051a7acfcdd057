"""FP64 quadrature of the Dirichlet Green function of the unit disk and the
unit ball over Voronoi cells (a checker for the oracle's binned estimators;
no part of the oracle or of the GPU path).

For Brownian motion with generator Lap/2 killed on leaving the unit ball
B in R^d, the occupation density is G(x, y) = 2 G_{-Lap}(x, y), with
Q(x, y) = |x|^2 |y|^2 - 2 x.y + 1 (= |x|^2 |y - x/|x|^2|^2, the image
point term):
  d = 2:  G = (1 / (2 pi)) ln(Q / |x - y|^2),
  d = 3:  G = (1 / (2 pi)) (|x - y|^-1 - Q^-1/2).
U f(x) = int G(x, y) f(y) dy and grad U f(x) = int grad_x G(x, y) f(y) dy
(Prop. "U_0 and DU_0" and the appendix lemma on the Green function of a
ball give the same kernel for the ball B(x, r) the walk steps through).

cell_integrals(x, centres) returns, for every Voronoi cell V_j of the
centres (nearest centre, Euclidean), int_{V_j cap B} G(x, y) dy and
int_{V_j cap B} grad_x G(x, y) dy, in polar (d = 2) or spherical (d = 3)
coordinates around x: along each ray x + rho e the cell V_j is one interval
of rho (the nearest-centre conditions are linear in rho), found exactly,
and integrated by Gauss-Legendre (with rho = s^2 on the interval that
starts at the singular point rho = 0).
"""
import numpy as np
from numpy.polynomial.legendre import leggauss


def green(x, y):
    d = x.shape[-1]
    xx = np.sum(x * x, -1)
    yy = np.sum(y * y, -1)
    xy = np.sum(x * y, -1)
    Q = xx * yy - 2.0 * xy + 1.0
    r2 = np.sum((x - y) ** 2, -1)
    if d == 2:
        return np.log(Q / r2) / (2.0 * np.pi)
    return (1.0 / np.sqrt(r2) - 1.0 / np.sqrt(Q)) / (2.0 * np.pi)


def grad_green(x, y):
    d = x.shape[-1]
    xx = np.sum(x * x, -1)
    yy = np.sum(y * y, -1)
    xy = np.sum(x * y, -1)
    Q = (xx * yy - 2.0 * xy + 1.0)[..., None]
    diff = x - y
    r2 = np.sum(diff * diff, -1)[..., None]
    img = yy[..., None] * x - y
    if d == 2:
        return (img / Q - diff / r2) / np.pi
    return (img / Q ** 1.5 - diff / r2 ** 1.5) / (2.0 * np.pi)


def _directions(d, n_dir):
    if d == 2:
        th = 2.0 * np.pi * (np.arange(n_dir) + 0.5) / n_dir
        return np.stack([np.cos(th), np.sin(th)], 1), np.full(n_dir, 2.0 * np.pi / n_dir)
    n_mu = int(round(np.sqrt(n_dir / 2.0)))
    n_ps = 2 * n_mu
    mu, wmu = leggauss(n_mu)
    ps = 2.0 * np.pi * (np.arange(n_ps) + 0.5) / n_ps
    M, P = np.meshgrid(mu, ps, indexing="ij")
    s = np.sqrt(1.0 - M * M)
    e = np.stack([s * np.cos(P), s * np.sin(P), M], -1).reshape(-1, 3)
    w = (wmu[:, None] * np.full(n_ps, 2.0 * np.pi / n_ps)[None, :]).reshape(-1)
    return e, w


def cell_integrals(x, centres, n_dir=4096, n_gl=24, chunk=512):
    """(m,) cell integrals of G(x, .) and (d, m) of grad_x G(x, .) over the
    Voronoi cells of `centres` intersected with the unit disk/ball."""
    x = np.asarray(x, dtype=np.float64)
    c = np.asarray(centres, dtype=np.float64)
    d = len(x)
    m = len(c)
    e_all, w_all = _directions(d, n_dir)
    s, ws = leggauss(n_gl)
    s = 0.5 * (s + 1.0)
    ws = 0.5 * ws
    dx = x - c
    nrm = np.sum(dx * dx, 1)
    a = nrm[:, None] - nrm[None, :]                     # a[j, k]
    A_out = np.zeros(m)
    B_out = np.zeros((d, m))
    for c0 in range(0, len(e_all), chunk):
        e = e_all[c0:c0 + chunk]
        w = w_all[c0:c0 + chunk]
        ex = e @ x
        rho_max = -ex + np.sqrt(ex * ex + 1.0 - x @ x)
        ey = e @ c.T                                       # (R, m)
        b = 2.0 * (ey[:, None, :] - ey[:, :, None])        # b[r, j, k] = 2 e.(c_k - c_j)
        # a[j,k] + rho b[r,j,k] <= 0 for every k
        with np.errstate(divide="ignore", invalid="ignore"):
            t = -a[None] / b
        lo = np.max(np.where(b < 0, t, -np.inf), axis=2)
        hi = np.min(np.where(b > 0, t, np.inf), axis=2)
        bad = np.any((b == 0) & (a[None] > 0), axis=2)
        lo = np.maximum(lo, 0.0)
        hi = np.minimum(hi, rho_max[:, None])
        hi = np.where(bad | (hi < lo), lo, hi)
        L = hi - lo                                        # (R, m)
        at0 = lo == 0.0
        # nodes: rho = lo + L s (plain) or lo + L s^2 (from the singular end)
        rho = np.where(at0[..., None], lo[..., None] + L[..., None] * s * s, lo[..., None] + L[..., None] * s)
        jac = np.where(at0[..., None], 2.0 * L[..., None] * s * ws, L[..., None] * ws)
        y = x + rho[..., None] * e[:, None, None, :]       # (R, m, g, d)
        xb = np.broadcast_to(x, y.shape)
        wt = jac * rho ** (d - 1) * w[:, None, None]
        ok = L[..., None] > 0
        with np.errstate(divide="ignore", invalid="ignore"):
            G = np.where(ok, green(xb, y), 0.0)
            dG = np.where(ok[..., None], grad_green(xb, y), 0.0)
        A_out += np.sum(G * wt, axis=(0, 2))
        B_out += np.einsum("rjga,rjg->aj", dG, wt)
    return A_out, B_out
