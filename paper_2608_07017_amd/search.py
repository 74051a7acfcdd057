"""Landscape exploration by p-HiSD with restarts (Table "numerical
parameters" and the comment below it, example "semilinear").

A run is p-HiSD of index k from a start (fbar0, directions from the Hessian
there), in blocks of `block` iterations; between blocks the gradient norm
|grad J|_{2,V} is read.  Besides its end point a run keeps fbar_close: the
iterate at the deepest dip of the norm before its final descent, i.e. the
lowest local minimum of the checked norms that is followed by a rise to at
least `rise` times its value (the paper restarts there, with other indices,
when the trajectory seems to have passed near another saddle).  Solutions
are compared modulo the symmetries of the problem (an optional list of site
permutations): two converged runs are the same solution when some symmetry
maps one's values at the sites onto the other's to a relative `same_tol`.
"""
import numpy as np

from ._lib import WosError


def run(tb, f, g, k, eta, tau, fbar0, max_iter, tol, block=50, rise=10.0, precond="A"):
    """One p-HiSD run of index k in blocks; returns a dict with the end
    point (fbar, u at the sites), its norm, the iterations, whether it
    converged, and fbar_close (None without a dip)."""
    fbar = fbar0
    V = None
    norms, snaps = [], []
    it = 0
    conv = False
    u = None
    J = None
    error = None
    while it < max_iter:
        nb = min(block, max_iter - it)
        try:
            u, _, fb, Vt, info = tb.saddle(f, g, k, eta, tau, nb, fbar0=fbar, V0=V, precond=precond)
        except WosError as e:  # e.g. directions that lost M-independence: the run stops there
            error = str(e)
            break
        it += info["iters"]
        fbar, V = fb, Vt
        norms.append(info["grad_norm"])
        snaps.append(fb.clone())
        J = info["J"]
        if info["grad_norm"] <= tol:
            conv = True
            break
    nv = np.asarray(norms)
    best = find_dip(nv, rise)
    close = None if best is None else snaps[best]
    if not norms:
        return {"k": k, "eta": eta, "fbar": None, "u": None, "grad_norm": float("inf"), "iters": 0,
                "converged": False, "J": None, "fbar_close": None, "close_norm": None, "error": error}
    return {"k": k, "eta": eta, "fbar": fbar, "u": u.cpu().numpy(), "grad_norm": float(nv[-1]), "iters": it,
            "converged": conv, "J": J, "fbar_close": close,
            "close_norm": None if best is None else float(nv[best]), "error": error}


def find_dip(norms, rise=10.0):
    """Index of the lowest local minimum of a sequence of gradient norms that
    is followed by a rise to at least `rise` times its value, or None."""
    nv = np.asarray(norms, dtype=np.float64)
    best = None
    for i in range(1, len(nv) - 1):
        if nv[i] < nv[i - 1] and nv[i] <= nv[i + 1] and nv[i + 1:].max() >= rise * nv[i]:
            if best is None or nv[i] < nv[best]:
                best = i
    return best


def same_solution(u1, u2, perms, same_tol):
    """Whether u2 is u1 up to one of the site permutations (and rounding)."""
    s = max(np.linalg.norm(u1), np.linalg.norm(u2), 1e-300)
    for p in perms:
        if np.linalg.norm(u1[p] - u2) <= same_tol * s:
            return True
    return False


def distinct(runs, perms, same_tol=1e-3):
    """Indices of the converged runs that give essentially distinct
    solutions (the first run of each class)."""
    keep = []
    for i, r in enumerate(runs):
        if not r["converged"]:
            continue
        if not any(same_solution(runs[j]["u"], r["u"], perms, same_tol) for j in keep):
            keep.append(i)
    return keep


def square_symmetries(sites, lo=(0.0, 0.0), hi=(1.0, 1.0)):
    """The eight symmetries of the square [lo, hi] as permutations of the
    sites (sites mapped onto sites to 1e-9 of the side); requires a
    symmetric layout."""
    x = (np.asarray(sites, dtype=np.float64) - np.asarray(lo)) / (np.asarray(hi) - np.asarray(lo))
    maps = [lambda a, b: (a, b), lambda a, b: (1 - a, b), lambda a, b: (a, 1 - b), lambda a, b: (1 - a, 1 - b),
            lambda a, b: (b, a), lambda a, b: (1 - b, a), lambda a, b: (b, 1 - a), lambda a, b: (1 - b, 1 - a)]
    out = []
    for mp in maps:
        ya, yb = mp(x[:, 0], x[:, 1])
        y = np.stack([ya, yb], 1)
        d2 = ((y[:, None, :] - x[None, :, :]) ** 2).sum(-1)
        p = np.argmin(d2, axis=1)
        if np.sqrt(d2[np.arange(len(x)), p].max()) > 1e-9:
            raise ValueError("the site layout is not symmetric under the square's symmetries")
        out.append(p)
    return out


def semilinear_s8000_table(tb, f, g, max_iter, tol, block=50):
    """The runs of Table "numerical parameters" for example "semilinear" at
    s = 8000: Adam (alpha 10, fbar_0 = 1) for the minimum; p-HiSD with
    fbar_0 = 1000, tau = 10: k = 1..8 at eta = 20, k = 5 at eta = 5, k = 6, 7
    at eta = 80; then from fbar_close of the (k, eta) = (4, 20), (5, 20),
    (5, 5), (6, 20) runs: k = 2, 3, 5; 2, 3, 4, 6; 4; 5, 7 at eta 20, 20, 5,
    20.  Returns the list of runs (the Adam run first, with k = 0)."""
    _, _, fb, info = tb.minimize(f, g, 0.0, 10.0, max_iter, fbar0=1.0, energy="semilinear", tol=tol,
                                 check_every=block)
    u, _ = tb.apply(fb, g)
    runs = [{"k": 0, "eta": None, "fbar": fb, "u": u.cpu().numpy(), "grad_norm": info["grad_norm"],
             "iters": info["iters"], "converged": info["grad_norm"] <= tol, "J": info["J"], "fbar_close": None,
             "start": "adam"}]
    first = {}
    for k, eta in [(k, 20.0) for k in range(1, 9)] + [(5, 5.0), (6, 80.0), (7, 80.0)]:
        r = run(tb, f, g, k, eta, 10.0, 1000.0, max_iter, tol, block)
        r["start"] = "1000"
        runs.append(r)
        first[(k, eta)] = r
    for (k0, eta0), ks in (((4, 20.0), (2, 3, 5)), ((5, 20.0), (2, 3, 4, 6)), ((5, 5.0), (4,)), ((6, 20.0), (5, 7))):
        src = first[(k0, eta0)]
        if src["fbar_close"] is None:
            continue
        for k in ks:
            r = run(tb, f, g, k, eta0, 10.0, src["fbar_close"], max_iter, tol, block)
            r["start"] = "close(k=%d, eta=%g)" % (k0, eta0)
            runs.append(r)
    return runs
