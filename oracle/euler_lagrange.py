"""Euler-Lagrange route: minimisation of the discrete functional J (oracle).

Test infrastructure (see the package header); never imported by the
product path.

Sec. "Euler-Lagrange boundary value problems": for an energy
F(x, u, p) the problem is reduced to the unknown source fbar in R^m through
u ~ U f + H g, with the toolbox estimators in place of the operators
(eq. gradJ):

    J(fbar) = sum_i lambda_i F(x_i, u_i, p_i),
    u_i = [A fbar + H g~]_i,   p_i = B_i fbar + K_i g~,

and its gradient (the boxed formula after eq. min_el_discrete)

    grad J = A^T (lambda o dF/du) + sum_a B^(a)^T (lambda o dF/dp_a).

The energies built here are those of the paper's nonlinear examples: the
p-Laplace one of Sec. "Solving nonlinear elliptic PDEs" (eq. plaplace),
F = |p|^P / P - f u, so dF/du = -f and dF/dp = |p|^(P-2) p (taken as 0 at
p = 0, its limit for P > 1); the minimal surface one, F = sqrt(1 + |p|^2)
- f u (f = 0 in the paper); and the semilinear one of the Breuer-McKenna-
Plum example, F = |p|^2 / 2 - u^3 / 3 + f u (Lap u + u^2 = f); and the
weighted quadratic one of the example "elliptic div min", F = w (p.A p / 2
+ c u^2 / 2 - f u) with w = exp(-phi), whose Euler-Lagrange equation is
-div(A grad u) + (A grad phi).grad u + c u = f.

The minimiser is Adam as restated in the appendix on the optimisation of
J: m_j = beta1 m_{j-1} + (1 - beta1) grad, v_j = beta2 v_{j-1} +
(1 - beta2) grad^2 (elementwise), alpha_j = alpha sqrt(1 - beta2^j) /
(1 - beta1^j), fbar_j = fbar_{j-1} - alpha_j m_j / (sqrt(v_j) + eps), with
m_0 = v_0 = 0 and the paper's beta1 = 0.9, beta2 = 0.999, eps = 1e-10.

Readings:
* the stopping norm |grad J|_{2,V} = (sum_j lambda(V_j) [grad J]_j^2)^(1/2)
  is taken with the normalised cell weights lambda_j = |V_j| / |D| (the
  toolbox's V and W cells are the same Voronoi cells of the sites), i.e.
  the paper's norm divided by sqrt(|D|);
* the paper gives final gradient norms but no stopping rule: a run stops
  after max_iter iterations or once the norm is at most tol.

Saddle points (the semilinear example's several solutions) are searched
by p-HiSD, ``phisd``, with M = A (n = m) as the paper takes it; its
initial directions are the eigenvectors of the k smallest eigenvalues of
the Hessian at fbar_0 (``semilinear_hessian``).  Reading: with M not
symmetric the M-orthonormalisation uses x^T M y with the left factor as in
the projections v v^T M.

``interpolate`` evaluates a solution off the sites, piecewise constant on
the cells or with the first-order correction <grad u_i, x - x_i>.

Pinned by tests/test_oracle_euler_lagrange.py:
* the gradient of every energy against central differences of J;
* the semilinear gradient against the regrouped sums Lambda0 fbar +
  Sigma0 g + A^T (lambda (f - u^2));
* the weighted quadratic gradient against the linear system of
  eq. linear_q with the coefficients (w A, 0, w c);
* the minimal surface gradient at small slope against the quadratic one;
* Adam's first step (of length alpha in every coordinate, a closed form of
  the update), and Adam on a separable quadratic against its known
  minimiser;
* the route at P = 2 against the linear system of eq. linear_q (the two
  routes of the paper coincide for the quadratic energy);
* the disk's closed-form p-torsion solution against the radial p-Laplace
  equation, and at P = 2 against (1 - |x|^2) / 4;
* p-HiSD on quadratics with a known saddle: the fixed point H^-1 b, with
  the directions spanning the unstable eigenvectors (M = I and an SPD M);
* the M-orthonormalisation for a non-symmetric M, and the QR factor for
  M = I;
* the semilinear Hessian against differences of the gradient;
* the interpolation, which reproduces affine fields exactly and returns
  u_i at the sites.
"""
import numpy as np

from .linalg import reconstruct


ENERGIES = ("plaplace", "minimal_surface", "semilinear", "elliptic")


def energy_parts(energy, tb, fbar, g, P, f, coef=None):
    """u, grad u (d, n), the energy density F_i and the weights
    (dF/du, dF/dp) at the sites for the energies of the paper's examples:
    "plaplace"         F = |p|^P / P - f u                (eq. plaplace)
    "minimal_surface"  F = sqrt(1 + |p|^2) - f u          (Example "minimal
                                                           surface", f = 0)
    "semilinear"       F = |p|^2 / 2 - u^3 / 3 + f u      (Example
                                                           "semilinear": Lap u + u^2 = f)
    "elliptic"         F = w (p.A p / 2 + c u^2 / 2 - f u) (Example
                       "elliptic div min", w = exp(-phi): -div(A grad u)
                       + (A grad phi).grad u + c u = f)
    (P is used by "plaplace" only; coef = {"A": (n, d, d), "c": (n,),
    "w": (n,)} by "elliptic", each optional: identity, 0, 1)."""
    u, gu = reconstruct(tb, fbar, g)
    s = np.sum(gu * gu, axis=0)  # |p_i|^2
    if energy == "plaplace":
        F = np.power(s, 0.5 * P) / P - f * u
        c = np.where(s > 0.0, np.power(np.where(s > 0.0, s, 1.0), 0.5 * (P - 2.0)), 0.0)  # |p|^(P-2)
        return u, gu, F, -f, c * gu
    if energy == "minimal_surface":
        q = np.sqrt(1.0 + s)
        return u, gu, q - f * u, -f, gu / q
    if energy == "semilinear":
        return u, gu, 0.5 * s - u ** 3 / 3.0 + f * u, f - u * u, gu
    if energy == "elliptic":
        coef = coef or {}
        n, d = u.shape[0], gu.shape[0]
        w = np.asarray(coef["w"], dtype=np.float64) if coef.get("w") is not None else np.ones(n)
        c = np.asarray(coef["c"], dtype=np.float64) if coef.get("c") is not None else np.zeros(n)
        Ac = (np.asarray(coef["A"], dtype=np.float64) if coef.get("A") is not None
              else np.broadcast_to(np.eye(d), (n, d, d)))
        Ap = np.einsum("nab,bn->an", Ac, gu)  # A_i p_i
        F = w * (0.5 * np.sum(gu * Ap, axis=0) + 0.5 * c * u * u - f * u)
        return u, gu, F, w * (c * u - f), w * Ap
    raise ValueError("unknown energy %r" % energy)


def plaplace_energy_parts(tb, fbar, g, P, f):
    """The parts of energy_parts for F = |p|^P / P - f u."""
    return energy_parts("plaplace", tb, fbar, g, P, f)


def energy_J(energy, tb, lam, fbar, g, P, f, coef=None):
    """J(fbar) = sum_i lambda_i F_i   (eq. gradJ)."""
    _, _, F, _, _ = energy_parts(energy, tb, fbar, g, P, f, coef)
    return float(np.sum(lam * F))


def energy_grad(energy, tb, lam, fbar, g, P, f, coef=None):
    """grad J = A^T (lambda o dF/du) + sum_a B^(a)^T (lambda o dF/dp_a)."""
    _, _, _, dFu, dFp = energy_parts(energy, tb, fbar, g, P, f, coef)
    grad = tb["A"].T @ (lam * dFu)
    for a in range(tb["B"].shape[0]):
        grad = grad + tb["B"][a].T @ (lam * dFp[a])
    return grad


def plaplace_J(tb, lam, fbar, g, P, f):
    """J(fbar) = sum_i lambda_i (|p_i|^P / P - f_i u_i)   (eq. gradJ)."""
    _, _, F, _, _ = plaplace_energy_parts(tb, fbar, g, P, f)
    return float(np.sum(lam * F))


def plaplace_grad(tb, lam, fbar, g, P, f):
    """grad J = A^T (lambda o dF/du) + sum_a B^(a)^T (lambda o dF/dp_a)."""
    _, _, _, dFu, dFp = plaplace_energy_parts(tb, fbar, g, P, f)
    grad = tb["A"].T @ (lam * dFu)
    for a in range(tb["B"].shape[0]):
        grad = grad + tb["B"][a].T @ (lam * dFp[a])
    return grad


def grad_norm(lam, grad):
    """(sum_j lambda_j grad_j^2)^(1/2) with the normalised cell weights."""
    return float(np.sqrt(np.sum(lam * grad * grad)))


def adam(grad_fn, f0, alpha, max_iter, beta1=0.9, beta2=0.999, eps=1e-10, tol=0.0, norm_fn=None,
         check_every=1):
    """Adam from f0 for at most max_iter iterations; with tol > 0 it stops
    after iteration j (a multiple of check_every) once norm_fn(grad J(f_j))
    <= tol.  Returns (f, iterations taken)."""
    f = np.array(f0, dtype=np.float64)
    m = np.zeros_like(f)
    v = np.zeros_like(f)
    j = 0
    for j in range(1, max_iter + 1):
        gr = grad_fn(f)
        m = beta1 * m + (1.0 - beta1) * gr
        v = beta2 * v + (1.0 - beta2) * gr * gr
        aj = alpha * np.sqrt(1.0 - beta2 ** j) / (1.0 - beta1 ** j)
        f = f - aj * m / (np.sqrt(v) + eps)
        if tol > 0.0 and j % check_every == 0 and norm_fn(grad_fn(f)) <= tol:
            break
    return f, j


def minimize_energy(energy, tb, lam, f, g, P, alpha, max_iter, f0=1.0, tol=0.0, check_every=1, lam_v=None,
                    coef=None):
    """Adam on J for any of the energies, from a constant fbar_0 = f0; the
    stopping norm uses lam_v (the V cells' measures; lam when None)."""
    m = tb["A"].shape[1]
    lv = lam if lam_v is None else lam_v
    fb, it = adam(lambda x: energy_grad(energy, tb, lam, x, g, P, f, coef), np.full(m, float(f0)), alpha, max_iter,
                  tol=tol, norm_fn=lambda gr: grad_norm(lv, gr), check_every=check_every)
    u, gu = reconstruct(tb, fb, g)
    return {"fbar": fb, "u": u, "grad_u": gu, "iters": it, "J": energy_J(energy, tb, lam, fb, g, P, f, coef),
            "grad_norm": grad_norm(lv, energy_grad(energy, tb, lam, fb, g, P, f, coef))}


def minimize_plaplace(tb, lam, f, g, P, alpha, max_iter, f0=1.0, tol=0.0, check_every=1):
    """The p-Laplace route end to end: Adam from fbar_0 = f0 (a constant,
    as in the paper's parameter table), then u, grad u, J and the norm."""
    m = tb["A"].shape[1]
    fb0 = np.full(m, float(f0))
    fb, it = adam(lambda x: plaplace_grad(tb, lam, x, g, P, f), fb0, alpha, max_iter, tol=tol,
                  norm_fn=lambda gr: grad_norm(lam, gr), check_every=check_every)
    u, gu = reconstruct(tb, fb, g)
    return {"fbar": fb, "u": u, "grad_u": gu, "iters": it, "J": plaplace_J(tb, lam, fb, g, P, f),
            "grad_norm": grad_norm(lam, plaplace_grad(tb, lam, fb, g, P, f))}


def semilinear_hessian(tb, lam, fbar, g):
    """The Hessian of J for F = |p|^2 / 2 - u^3 / 3 + f u:
    H = sum_a B^(a)^T diag(lambda) B^(a) + A^T diag(lambda (-2 u)) A
    (d2F/dp2 = I, d2F/du2 = -2u, no mixed term)."""
    u, _ = reconstruct(tb, fbar, g)
    H = tb["A"].T @ ((lam * (-2.0 * u))[:, None] * tb["A"])
    for a in range(tb["B"].shape[0]):
        H = H + tb["B"][a].T @ (lam[:, None] * tb["B"][a])
    return H


def m_orthonormalize(V, M):
    """Gram-Schmidt of the columns v_1..v_k of V in the form <x, y>_M =
    x^T M y (the form of the projections v v^T M of p-HiSD):
    v_i <- v_i - sum_{l<i} <v_l, v_i>_M v_l, then v_i / <v_i, v_i>_M^(1/2)."""
    V = np.array(V, dtype=np.float64)
    for i in range(V.shape[1]):
        for l in range(i):
            V[:, i] -= (V[:, l] @ (M @ V[:, i])) * V[:, l]
        V[:, i] /= np.sqrt(V[:, i] @ (M @ V[:, i]))
    return V


def phisd(grad_fn, f0, V0, M, eta, tau, max_iter, tol=0.0, norm_fn=None, check_every=1):
    """Preconditioned high-index saddle dynamics (p-HiSD), as the paper
    states it in its appendix on the optimisation of J: from fbar_0 and k
    directions V^(0) (M-orthonormalised first), for j >= 1
      fbar_j = fbar_{j-1} - eta R M^-1 grad J(fbar_{j-1}),
               R = I - 2 sum_i v_i v_i^T M,
      v_i   <- v_i - tau P_i M^-1 H(fbar_j) v_i,
               P_i = I - v_i v_i^T M - 2 sum_{l<i} v_l v_l^T M,
    all with the previous V, then V M-orthonormalised; H(fbar) v is the
    central difference (grad J(fbar + h v) - grad J(fbar - h v)) / (2h),
    h = 1e-6 max(1, |fbar|_2).  With tol > 0 the run stops after iteration
    j (a multiple of check_every) once norm_fn(grad J(fbar_j)) <= tol.
    Returns (fbar, V, iterations taken)."""
    f = np.array(f0, dtype=np.float64)
    V = m_orthonormalize(V0, M)
    k = V.shape[1]
    j = 0
    for j in range(1, max_iter + 1):
        w = np.linalg.solve(M, grad_fn(f))
        Rw = w - 2.0 * sum(V[:, i] * (V[:, i] @ (M @ w)) for i in range(k))
        f = f - eta * Rw
        h = 1e-6 * max(1.0, float(np.linalg.norm(f)))
        Vn = V.copy()
        for i in range(k):
            Hv = (grad_fn(f + h * V[:, i]) - grad_fn(f - h * V[:, i])) / (2.0 * h)
            y = np.linalg.solve(M, Hv)
            Py = y - V[:, i] * (V[:, i] @ (M @ y))
            for l in range(i):
                Py = Py - 2.0 * V[:, l] * (V[:, l] @ (M @ y))
            Vn[:, i] = V[:, i] - tau * Py
        V = m_orthonormalize(Vn, M)
        if tol > 0.0 and j % check_every == 0 and norm_fn(grad_fn(f)) <= tol:
            break
    return f, V, j


def interpolate(sites, u, grad_u, x):
    """Evaluation off the sites (the approximations after eq.
    min_el_discrete): for x in the cell W_i of its nearest site x_i,
    u(x) ~ u_i + <grad u_i, x - x_i> (the gradient-enhanced form), or u_i
    when grad_u is None (piecewise constant).  Returns (values, i)."""
    from .voronoi import nearest
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    i = nearest(sites, x)
    v = np.asarray(u, dtype=np.float64)[i].copy()
    if grad_u is not None:
        gu = np.asarray(grad_u, dtype=np.float64)
        v += np.sum(gu[:, i].T * (x - np.asarray(sites, dtype=np.float64)[i]), axis=1)
    return v, i


def plaplace_torsion_disk(x, P):
    """The disk's p-torsion solution (-Lap_p u = 1, u = 0 on the circle),
    Example "p-Torsion problem on unit disk":
    u = (P-1)/P (1/2)^(1/(P-1)) (1 - |x|^(P/(P-1)))."""
    r2 = np.sum(np.asarray(x, dtype=np.float64) ** 2, axis=-1)
    return (P - 1.0) / P * 0.5 ** (1.0 / (P - 1.0)) * (1.0 - np.power(r2, P / (2.0 * P - 2.0)))
