"""Reduction of a Dirichlet problem to the system for the unknown source (oracle).

Sec. "Second order linear elliptic PDEs": for
    L u = div(A grad u) + b . grad u - c u = f in D,  u = g on the boundary
(eq. linearPDE, the paper's sign convention), the ansatz u ~ U q + H g,
Galerkin testing with U phi and the cell-centre quadrature of Rem.
"discretization" give (eq. linear_q)

    Lambda q = -(A^lambda)^T f~ - Sigma g~,
    Lambda = sum_i lambda_i B_i^T A(x_i) B_i - A^T B^b + A^T diag(lambda c~) A,
    Sigma  = sum_i lambda_i B_i^T A(x_i) K_i - A^T K^b + A^T H^c,

with B_i = (B^(k)_{ij})_{k,j} (d x m), K_i likewise, B^b_{ij} =
lambda_i <B_{.ij}, b(x_i)>, K^b likewise, H^c_{ij} = lambda_i c_i H_{ij};
then u = A q + H g~ and grad u_i = B_i q + K_i g~ (the boxed
reconstruction; Sec. "Euler-Lagrange" for the gradient).

Readings taken here:
* the right-hand side term "A^lambda f~" is dimensionally (n x m)(n,) and is
  read as (A^lambda)^T f~ = A^T (lambda o f~), which is what the derivation
  above it produces (sum_i lambda_i f(x_i) [A phi]_i);
* the generalised inverse is the truncated SVD: singular values <= rcond *
  sigma_max are dropped (the paper's TSVD, default rcond 1e-3);
* sum_i lambda_i B_i^T A(x_i) B_i is evaluated as
  sum_{a,b} B^(a)^T diag(lambda A_ab) B^(b), the same sum regrouped so that
  library matrix products do the work.

Nonlinear outer loops (not in the paper; the paper uses Adam / HiSD on the
discrete functional J of eq. gradJ):
* Newton for -Lap u + kappa u^3 = f: J(h) = sum_i lambda_i F(u_i, p_i) with
  F = |p|^2/2 + kappa u^4/4 - f u, u = A h + H g, p_i = B_i h + K_i g;
  grad J = A^T (lambda o (kappa u^3 - f)) + Lambda0 h + Sigma0 g (the boxed
  gradient of Sec. "Euler-Lagrange"), Hessian = Lambda0 + A^T diag(3 kappa
  lambda u^2) A, with Lambda0 = sum_i lambda_i B_i^T B_i.
* Picard for -div((1 + u^2) grad u) = f: each iterate solves eq. linear_q
  with A(x_i) = (1 + u_i^2) I, b = 0, c = 0 and the paper's f = -f.

Pinned by tests/test_oracle_linalg.py: the regrouped sums against the
literal per-cell sums, the TSVD against numpy's SVD pseudo-inverse, the
Newton iteration on the quadratic energy against the linear system (the two
routes of the paper coincide), end-to-end errors against manufactured
solutions on the unit disk, and the Picard fixed point against the
Kirchhoff transform w = u + u^3/3 of the same problem (a linear solve for w).
"""
import numpy as np


def _grad_pairs(B, K, lam, Acoef):
    """sum_i lambda_i B_i^T A(x_i) B_i and sum_i lambda_i B_i^T A(x_i) K_i."""
    d, n, m = B.shape
    p = K.shape[2]
    L = np.zeros((m, m))
    S = np.zeros((m, p))
    for a in range(d):
        for b in range(d):
            wab = lam * (Acoef[:, a, b] if Acoef is not None else (1.0 if a == b else 0.0))
            if np.all(wab == 0):
                continue
            L += B[a].T @ (wab[:, None] * B[b])
            S += B[a].T @ (wab[:, None] * K[b])
    return L, S


def assemble(tb, lam, Acoef=None, bcoef=None, ccoef=None):
    """Lambda (m x m) and Sigma (m x p) of eq. linear_q.

    Acoef: (n,d,d) or None (identity); bcoef: (n,d) or None; ccoef: (n,) or None.
    """
    A, B, H, K = tb["A"], tb["B"], tb["H"], tb["K"]
    lam = np.asarray(lam, dtype=np.float64)
    L, S = _grad_pairs(B, K, lam, Acoef)
    if bcoef is not None:
        Bb = lam[:, None] * np.einsum("na,anm->nm", bcoef, B)
        Kb = lam[:, None] * np.einsum("na,anp->np", bcoef, K)
        L -= A.T @ Bb
        S -= A.T @ Kb
    if ccoef is not None:
        lc = lam * ccoef
        L += A.T @ (lc[:, None] * A)
        S += A.T @ (lc[:, None] * H)
    return L, S


def rhs(tb, lam, Sigma, f, g):
    """-(A^lambda)^T f~ - Sigma g~, with f the paper's right-hand side (L u = f)."""
    return -tb["A"].T @ (lam * f) - Sigma @ g


def tsvd_solve(M, r, rcond):
    """Truncated-SVD solution: singular values <= rcond * sigma_max dropped."""
    U, s, Vt = np.linalg.svd(M)
    keep = s > rcond * s[0]
    return Vt[keep].T @ ((U[:, keep].T @ r) / s[keep])


def tikhonov_solve(M, r, rcond):
    """Tikhonov-regularised generalised inverse (a regularised inverse in the
    sense of the paper's solve step): q minimises |M q - r|^2 + reg |q|^2 with
    reg = rcond^2 max_j (M^T M)_jj, i.e. (M^T M + reg I) q = M^T r.
    Returns (q, reg)."""
    N = M.T @ M
    reg = rcond * rcond * float(np.max(np.diag(N)))
    return np.linalg.solve(N + reg * np.eye(N.shape[0]), M.T @ r), reg


def sym_reg_solve(M, r, rcond):
    """Regularised solve of a symmetric positive semidefinite system:
    (M + reg I)^{-1} r with reg = rcond max_j M_jj."""
    reg = rcond * float(np.max(np.diag(M)))
    return np.linalg.solve(M + reg * np.eye(M.shape[0]), r), reg


def reconstruct(tb, q, g):
    """u = A q + H g~ and grad u (d, n)."""
    u = tb["A"] @ q + tb["H"] @ g
    gu = np.einsum("anm,m->an", tb["B"], q) + np.einsum("anp,p->an", tb["K"], g)
    return u, gu


def solve_linear(tb, lam, f, g, Acoef=None, bcoef=None, ccoef=None, rcond=1e-3, solver="tsvd"):
    L, S = assemble(tb, lam, Acoef, bcoef, ccoef)
    if solver == "tikhonov":
        q, _ = tikhonov_solve(L, rhs(tb, lam, S, f, g), rcond)
    else:
        q = tsvd_solve(L, rhs(tb, lam, S, f, g), rcond)
    u, gu = reconstruct(tb, q, g)
    return {"q": q, "u": u, "grad_u": gu, "Lambda": L, "Sigma": S}


def apply_direct(tb, fbar, g):
    """Known source: u = A fbar + H g (-(1/2) Lap u = fbar), and its gradient."""
    return reconstruct(tb, fbar, g)


def _sym_step(M, r, rcond, solver):
    return tsvd_solve(M, r, rcond) if solver == "tsvd" else sym_reg_solve(M, r, rcond)[0]


def newton(tb, lam, g, dFu, d2Fu, rcond=1e-3, tol=1e-8, max_iter=50, h0=None, solver="tsvd"):
    """Newton on grad J = 0 for F(x, u, p) = |p|^2/2 + G(x, u), with
    dFu(u) = dG/du and d2Fu(u) = d^2G/du^2 at the sites."""
    A, H = tb["A"], tb["H"]
    L0, S0 = _grad_pairs(tb["B"], tb["K"], lam, None)
    h = np.zeros(A.shape[1]) if h0 is None else np.array(h0, dtype=np.float64)
    gnorm0 = None
    it = 0
    for it in range(max_iter + 1):
        u = A @ h + H @ g
        grad = A.T @ (lam * dFu(u)) + L0 @ h + S0 @ g
        gn = np.linalg.norm(grad)
        if gnorm0 is None:
            gnorm0 = gn
        if gn <= tol * gnorm0 or it == max_iter:
            break
        hess = L0 + A.T @ ((lam * d2Fu(u))[:, None] * A)
        h = h - _sym_step(hess, grad, rcond, solver)
    u, gu = reconstruct(tb, h, g)
    return {"h": h, "u": u, "grad_u": gu, "iters": it, "grad_norm": gn, "grad_norm0": gnorm0}


def newton_cubic(tb, lam, f, g, kappa=1.0, rcond=1e-3, tol=1e-8, max_iter=50, solver="tsvd"):
    """Newton for -Lap u + kappa u^3 = f (F = |p|^2/2 + kappa u^4/4 - f u),
    started at the solution of the problem without the cubic term."""
    A = tb["A"]
    L0, S0 = _grad_pairs(tb["B"], tb["K"], lam, None)
    h0 = _sym_step(L0, A.T @ (lam * f) - S0 @ g, rcond, solver)
    return newton(tb, lam, g, dFu=lambda u: kappa * u ** 3 - f, d2Fu=lambda u: 3.0 * kappa * u * u,
                  rcond=rcond, tol=tol, max_iter=max_iter, h0=h0, solver=solver)


def picard_quasilinear(tb, lam, f, g, rcond=1e-3, tol=1e-10, max_iter=100, solver="tsvd"):
    """Picard for -div((1+u^2) grad u) = f: A(x_i) = (1 + u_i^2) I, paper f = -f."""
    d, n, _ = tb["B"].shape
    u = np.zeros(n)
    it = 0
    for it in range(1, max_iter + 1):
        a = 1.0 + u * u
        Acoef = a[:, None, None] * np.eye(d)[None]
        res = solve_linear(tb, lam, -f, g, Acoef=Acoef, rcond=rcond, solver=solver)
        un = res["u"]
        du = np.sqrt(np.sum(lam * (un - u) ** 2))
        nu = np.sqrt(np.sum(lam * un ** 2))
        u = un
        if du <= tol * nu:
            break
    res["iters"] = it
    return res
