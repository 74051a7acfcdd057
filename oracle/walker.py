"""The Walk-on-Spheres toolbox estimators (oracle, FP64).

Follows Alg. "WoS-LOT" (Sec. "Laplacian Operator Toolbox: Pseudocode
algorithms"), which builds A, B^(j), H, K^(j) in one pass per walk, in the
refined form of Rem. "MC_no_singular" (samplers in ``oracle.samplers``).
For site x = x_i and walk l, with r0 = r(x):

1. per-walk draws: R ~ Beta(2,2), Z, Zs, U1 uniform on the sphere, S;
   Y = R Z; omega (d = 2 only, else 1) -- or, with sampler="lambert" in
   d = 2, R from the exact radial law (the Lambert W form of Prop.
   "removing singularities" (i.1), from the first of the same uniforms)
   and omega = 1; w = (d / r0) U1 (the factor
   (X_1 - x) d / r0^2 of eqs. Estimator_B and Estimator_K);
2. ball term of eq. Estimator_B, refined: tally r0 * sum_{k<d} S^k * Zs
   into B at the cell of x + r0 S Zs;
3. the k = 0 term of eq. Estimator_A: tally omega r0^2 / d into A at the
   cell of x + r0 Y (B's chain term starts at s = 1);
4. first step X_1 = x + r0 U1 (eq. wos chain);
5. for k = 1, 2, ...: r = r(X_k); stop if r < eps (or k > max_steps);
   t = omega r^2 / d; tally t into A and t * w into B at the cell of
   X_k + r Y; move X_{k+1} = X_k + r U_k;
6. terminal point X_T: count 1 into H and add w into K at its boundary
   cell (eqs. Estimator_H, Estimator_K);
7. divide by N.

Readings of the paper taken here:
* the paper runs a fixed number M of steps; the default here stops at the
  first k >= 1 with r(X_k) < eps (``fixed_M > 0`` gives the paper's rule:
  exactly M chain tallies, terminal point X_{M+1} as in Alg. "WoS-LOT");
* the terminal point is binned as is, without projection on the boundary;
* every (site, walk) pair draws its own random numbers (the estimator
  definitions use i.i.d. copies per x and l; the pseudocode's sharing of
  one draw across all sites is not reproduced);
* Y is drawn once per walk and reused at every step, by A and by B.

Walks are simulated together as arrays (the paper's Rem.
"implementation_tips" (ii) vectorises over walks); each walk's arithmetic
is exactly the steps above.

The V cells (the columns of A and B) may be a partition of their own
(Rem. after the definition of the partitions: W_n and V_m chosen
independently); with ``vcentres`` the tally points are binned to those
centres, the walks themselves are unchanged.

Pinned by tests/test_oracle_green_pins.py: every entry of A and B of a
row against the disk's and the ball's Green function integrated over the
Voronoi cells (and its gradient in x), the pointwise estimators of
non-harmonic defining functions (U(-Lap phi / 2) = phi and its gradient)
on the disk, ball, square, L-shape and cube minus ball, the harmonic
extension of |y| on the disk with its gradient, and the square's torsion
function; tests/test_oracle_mutations.py checks that these pins fail for
copies of this file with one plausible mistake planted (tally point,
k = 0 point, ball term, omega, signs, terminal point, K weight).
Pinned by tests/test_oracle_walker.py: E tau = (1-|x|^2)/d and its
gradient on the unit disk and ball (eps bias bounded by 2 eps / d), the
closed forms U[x_1] and grad U[x_1], the harmonic extension and its
gradient for harmonic boundary data, the disk's harmonic measure of an arc,
H row sums equal to 1, and the binned matrices against the same walks'
pointwise estimators on piecewise-constant data; with a separate V
partition, the row sums unchanged and the columns permuted with the
centres.
"""
import numpy as np

from .geometry import distance
from .philox import walk_block, step_uniforms
from .samplers import median3, omega, s_of_u, ball_weight_poly, sphere, lambert_radius
from .voronoi import nearest

DEFAULT_MAX_STEPS = 10000


class SiteEvents:
    """Everything the walks of one site tally, before binning.

    ball_pts (N,d), ball_w (N,d): ball term of B.
    ev_walk (E,), ev_pts (E,d), ev_tA (E,), ev_tB (E,d): the k >= 0 chain
    tallies (A weight and B weight, the k = 0 one has zero B weight).
    term_pts (N,d), term_w (N,d): terminal point and K weight per walk.
    nsteps (N,): walk-steps per walk (the k = 0 tally plus chain tallies).
    capped (N,): walks stopped by the step cap.
    """


def site_events(dom, x, i, walks, eps, seed, max_steps=DEFAULT_MAX_STEPS, fixed_M=0, sampler="median3"):
    d = dom["dim"]
    x = np.asarray(x, dtype=np.float64).reshape(d)
    l = np.asarray(walks, dtype=np.int64)
    N = len(l)
    r0 = float(distance(dom, x[None])[0])
    if not r0 > 0:
        raise ValueError("site outside the domain")

    b0 = walk_block(seed, l, i, 0)
    exact = sampler == "lambert"
    if exact and d != 2:
        raise ValueError("the Lambert W sampler is for d = 2")
    R = lambert_radius(b0[0]) if exact else median3(b0[0], b0[1], b0[2])
    S = s_of_u(b0[3])
    b1 = walk_block(seed, l, i, 1)
    if d == 2:
        Z = sphere(2, [b1[0]])
        Zs = sphere(2, [b1[1]])
        U1 = sphere(2, [b1[2]])
    else:
        b2 = walk_block(seed, l, i, 2)
        Z = sphere(3, [b1[0], b1[1]])
        Zs = sphere(3, [b1[2], b1[3]])
        U1 = sphere(3, [b2[0], b2[1]])
    om = np.ones_like(R) if exact else omega(R, d)
    Y = R[:, None] * Z
    w = (d / r0) * U1

    ev = SiteEvents()
    ev.ball_pts = x + r0 * S[:, None] * Zs
    ev.ball_w = r0 * ball_weight_poly(S, d)[:, None] * Zs

    walk_ids, pts, tA, tB = [np.arange(N)], [x + r0 * Y], [om * r0 * r0 / d], [np.zeros((N, d))]
    X = x + r0 * U1
    k = np.ones(N, dtype=np.int64)
    nsteps = np.ones(N, dtype=np.int64)
    capped = np.zeros(N, dtype=bool)
    alive = np.ones(N, dtype=bool)
    idx = np.arange(N)
    while True:
        a = idx[alive]
        if len(a) == 0:
            break
        r = distance(dom, X[a])
        if fixed_M > 0:
            stop = k[a] > fixed_M
            r = np.maximum(r, 0.0)
        else:
            near = r < eps
            over = k[a] > max_steps
            capped[a[over & ~near]] = True
            stop = near | over
        alive[a[stop]] = False
        a, r = a[~stop], r[~stop]
        if len(a) == 0:
            break
        t = om[a] * r * r / d
        walk_ids.append(a)
        pts.append(X[a] + r[:, None] * Y[a])
        tA.append(t)
        tB.append(t[:, None] * w[a])
        nsteps[a] += 1
        U = sphere(d, step_uniforms(seed, l[a], i, k[a], d))
        X[a] = X[a] + r[:, None] * U
        k[a] += 1

    ev.ev_walk = np.concatenate(walk_ids)
    ev.ev_pts = np.concatenate(pts)
    ev.ev_tA = np.concatenate(tA)
    ev.ev_tB = np.concatenate(tB)
    ev.term_pts = X
    ev.term_w = w
    ev.nsteps = nsteps
    ev.capped = capped
    ev.r0 = r0
    return ev


def bin_site(ev, sites, bnodes, m=None, p=None):
    """Bin one site's events: returns the unnormalised rows
    (A_row (m,), B_rows (d,m), Hcount_row (p,), K_rows (d,p))."""
    sites = np.asarray(sites, dtype=np.float64)
    bnodes = np.asarray(bnodes, dtype=np.float64)
    m = len(sites) if m is None else m
    p = len(bnodes) if p is None else p
    d = sites.shape[1]
    jv = nearest(sites, ev.ev_pts)
    jb = nearest(sites, ev.ball_pts)
    jg = nearest(bnodes, ev.term_pts)
    A_row = np.bincount(jv, weights=ev.ev_tA, minlength=m)
    B_rows = np.stack([np.bincount(jb, weights=ev.ball_w[:, a], minlength=m)
                       + np.bincount(jv, weights=ev.ev_tB[:, a], minlength=m) for a in range(d)])
    H_row = np.bincount(jg, minlength=p).astype(np.int64)
    K_rows = np.stack([np.bincount(jg, weights=ev.term_w[:, a], minlength=p) for a in range(d)])
    return A_row, B_rows, H_row, K_rows


def build_toolbox(dom, sites, bnodes, walks, eps, seed, max_steps=DEFAULT_MAX_STEPS,
                  fixed_M=0, rows=None, vcentres=None, sampler="median3"):
    """The toolbox A (n,m), B (d,n,m), H (n,p), K (d,n,p) of eq. LOT.

    Centres: W-centres = ``sites`` (the walks' starting points, n rows),
    V-centres = ``vcentres`` (the cells the tally points are binned to, m
    columns; the same as ``sites`` when None, n = m), Gamma-centres =
    ``bnodes``.  ``rows`` restricts the output to a subset of sites (rows
    are independent: each (site, walk) pair has its own random stream).
    """
    sites = np.asarray(sites, dtype=np.float64)
    bnodes = np.asarray(bnodes, dtype=np.float64)
    vc = sites if vcentres is None else np.asarray(vcentres, dtype=np.float64)
    n, d = sites.shape
    m = len(vc)
    p = len(bnodes)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    nr = len(rows)
    A = np.zeros((nr, m))
    B = np.zeros((d, nr, m))
    Hc = np.zeros((nr, p), dtype=np.int64)
    K = np.zeros((d, nr, p))
    steps = np.zeros(nr, dtype=np.int64)
    maxk = np.zeros(nr, dtype=np.int64)
    capped = np.zeros(nr, dtype=np.int64)
    for row, i in enumerate(rows):
        ev = site_events(dom, sites[i], int(i), np.arange(walks), eps, seed, max_steps, fixed_M, sampler)
        a_row, b_rows, h_row, k_rows = bin_site(ev, vc, bnodes)
        A[row] = a_row / walks
        B[:, row] = b_rows / walks
        Hc[row] = h_row
        K[:, row] = k_rows / walks
        steps[row] = ev.nsteps.sum()
        maxk[row] = ev.nsteps.max()
        capped[row] = ev.capped.sum()
    return {"A": A, "B": B, "H": Hc / walks, "Hcount": Hc, "K": K,
            "walk_steps": steps, "max_steps": maxk, "capped": capped, "rows": rows}


def pointwise(dom, x, i, walks, eps, seed, f=None, g=None, max_steps=DEFAULT_MAX_STEPS,
              fixed_M=0, sampler="median3"):
    """The pointwise estimators of Sec. "Monte Carlo estimators" in their
    refined form: U^f (eq. u MC), grad U^f (eq. gradu U MC), H^g (eq. H MC),
    grad H^g (eq. dh MC), each with its per-walk standard error.

    f: callable on points (k,d) -> (k,); g: callable on points -> (k,).
    Returns a dict of means and standard errors.
    """
    ev = site_events(dom, x, i, np.arange(walks), eps, seed, max_steps, fixed_M, sampler)
    N = walks
    d = dom["dim"]
    out = {"r0": ev.r0, "nsteps": ev.nsteps}

    def mean_se(per_walk):
        per_walk = np.asarray(per_walk)
        mu = per_walk.mean(axis=0)
        se = per_walk.std(axis=0, ddof=1) / np.sqrt(N)
        return mu, se

    if f is not None:
        fv = f(ev.ev_pts)
        cu = np.bincount(ev.ev_walk, weights=ev.ev_tA * fv, minlength=N)
        cg = np.stack([np.bincount(ev.ev_walk, weights=ev.ev_tB[:, a] * fv, minlength=N)
                       + ev.ball_w[:, a] * f(ev.ball_pts) for a in range(d)], axis=1)
        out["U"], out["U_se"] = mean_se(cu)
        out["gradU"], out["gradU_se"] = mean_se(cg)
    if g is not None:
        gv = g(ev.term_pts)
        out["H"], out["H_se"] = mean_se(gv)
        out["gradH"], out["gradH_se"] = mean_se(ev.term_w * gv[:, None])
    return out


def site_functionals(dom, x, i, walks, eps, seed, vcentres, bnodes, phi, psi, max_steps=DEFAULT_MAX_STEPS,
                     fixed_M=0, sampler="median3"):
    """The per-walk values of the four estimators of Sec. "Monte Carlo
    estimators" (eqs. u MC, gradu U MC, H MC, dh MC) with binned data: f is
    phi at the nearest V centre, g is psi at the nearest boundary centre.
    Returns (cA (N,), cB (N,d), cH (N,), cK (N,d)); their means are the rows
    A phi, B phi, H psi and K psi of the binned toolbox."""
    vc = np.asarray(vcentres, dtype=np.float64)
    bn = np.asarray(bnodes, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    ev = site_events(dom, x, i, np.arange(walks), eps, seed, max_steps, fixed_M, sampler)
    d = dom["dim"]
    f_ev = phi[nearest(vc, ev.ev_pts)]
    f_ball = phi[nearest(vc, ev.ball_pts)]
    g_term = psi[nearest(bn, ev.term_pts)]
    cA = np.bincount(ev.ev_walk, weights=ev.ev_tA * f_ev, minlength=walks)
    cB = np.stack([np.bincount(ev.ev_walk, weights=ev.ev_tB[:, a] * f_ev, minlength=walks)
                   + ev.ball_w[:, a] * f_ball for a in range(d)], axis=1)
    cH = g_term
    cK = ev.term_w * g_term[:, None]
    return cA, cB, cH, cK
