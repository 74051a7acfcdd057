"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module generates INPUTS only: domains, interior sites, boundary nodes,
coefficient fields and manufactured solutions.  It holds none of the
method's arithmetic (no distance to the boundary, no walks, no binning, no
assembly), and neither the oracle nor the GPU path is imported here.

Recipes (the paper publishes no data; shapes follow its experiments and the
benchmark configurations):

* sites: uniform in D by rejection from the bounding box with numpy's PCG64
  generator, keeping points whose distance to the boundary exceeds a margin
  (10 * eps by default, so that no site starts inside the stopping shell);
* the paper's deterministic layouts: the disk's rings r_k = (k - 1/2)/10
  with 6k - 3 points each (k = 1..10, n = 300) and 60 boundary nodes; the
  square's 20 x 20 cell centres with 20 boundary nodes per edge at the edge
  midpoints of the boundary cells (Sec. "Numerical examples", setup);
* boundary nodes: equispaced angles on the circle; (k + 1/2)/q on each edge
  of a box face; Fibonacci points on a sphere (z_k = 1 - (2k+1)/p,
  phi_k = k pi (3 - sqrt 5)); equispaced arc length along a polygon's edges;
  face-cell midpoints on the faces of a cube.
"""
import numpy as np

# ---------------------------------------------------------------- domains


def unit_disk():
    return {"kind": "ball", "dim": 2, "center": [0.0, 0.0], "radius": 1.0}


def unit_ball():
    return {"kind": "ball", "dim": 3, "center": [0.0, 0.0, 0.0], "radius": 1.0}


def unit_square():
    return {"kind": "box", "dim": 2, "lo": [0.0, 0.0], "hi": [1.0, 1.0]}


def l_shape():
    """(-1,1)^2 minus [0,1) x (-1,0], counter-clockwise (the paper's L-shape)."""
    verts = [[-1.0, -1.0], [0.0, -1.0], [0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [-1.0, 1.0]]
    return {"kind": "polygon", "dim": 2, "verts": verts}


def cube_minus_ball():
    return {"kind": "box_minus_ball", "dim": 3, "lo": [0.0, 0.0, 0.0], "hi": [1.0, 1.0, 1.0],
            "center": [0.5, 0.5, 0.5], "radius": 0.3}


# ------------------------------------------------- interior with a margin


def _box_gap(x, lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return np.minimum(x - lo, hi - x).min(axis=1)


def _outside_box_gap(x, lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    e = np.maximum(np.maximum(lo - x, x - hi), 0.0)
    return np.sqrt((e * e).sum(axis=1))


def interior_with_margin(dom, x, margin):
    """True where x lies in D at distance > margin from the boundary
    (written per workload domain; used only to draw inputs)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    k = dom["kind"]
    if k == "ball":
        c = np.asarray(dom["center"], dtype=np.float64)
        return np.linalg.norm(x - c, axis=1) < dom["radius"] - margin
    if k == "box":
        return _box_gap(x, dom["lo"], dom["hi"]) > margin
    if k == "polygon":
        if dom["verts"] != l_shape()["verts"]:
            raise ValueError("only the L-shape polygon has an input recipe")
        return (_box_gap(x, [-1, -1], [1, 1]) > margin) & \
            (_outside_box_gap(x, [0, -1], [1, 0]) > margin)
    if k == "box_minus_ball":
        c = np.asarray(dom["center"], dtype=np.float64)
        return (_box_gap(x, dom["lo"], dom["hi"]) > margin) & \
            (np.linalg.norm(x - c, axis=1) > dom["radius"] + margin)
    raise ValueError(k)


def bbox(dom):
    k = dom["kind"]
    d = dom["dim"]
    if k == "ball":
        c = np.asarray(dom["center"], dtype=np.float64)[:d]
        return c - dom["radius"], c + dom["radius"]
    if k == "polygon":
        v = np.asarray(dom["verts"], dtype=np.float64)
        return v.min(axis=0), v.max(axis=0)
    return np.asarray(dom["lo"], dtype=np.float64), np.asarray(dom["hi"], dtype=np.float64)


def sample_sites(dom, n, seed, margin):
    """n points uniform in {x in D : dist(x, boundary) > margin}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = bbox(dom)
    out = []
    have = 0
    while have < n:
        cand = lo + (hi - lo) * rng.random((max(64, 2 * (n - have)), dom["dim"]))
        cand = cand[interior_with_margin(dom, cand, margin)]
        out.append(cand)
        have += len(cand)
    return np.concatenate(out)[:n]


# --------------------------------------------------------- boundary nodes


def circle_nodes(p, center=(0.0, 0.0), radius=1.0):
    th = 2.0 * np.pi * np.arange(p) / p
    return np.stack([center[0] + radius * np.cos(th), center[1] + radius * np.sin(th)], axis=1)


def square_nodes(per_edge, lo=(0.0, 0.0), hi=(1.0, 1.0)):
    t = (np.arange(per_edge) + 0.5) / per_edge
    x0, y0 = lo
    x1, y1 = hi
    bottom = np.stack([x0 + (x1 - x0) * t, np.full(per_edge, y0)], axis=1)
    right = np.stack([np.full(per_edge, x1), y0 + (y1 - y0) * t], axis=1)
    top = np.stack([x1 - (x1 - x0) * t, np.full(per_edge, y1)], axis=1)
    left = np.stack([np.full(per_edge, x0), y1 - (y1 - y0) * t], axis=1)
    return np.concatenate([bottom, right, top, left])


def fibonacci_sphere(p, center=(0.0, 0.0, 0.0), radius=1.0):
    k = np.arange(p)
    z = 1.0 - (2.0 * k + 1.0) / p
    ph = k * np.pi * (3.0 - np.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    pts = np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)
    return np.asarray(center) + radius * pts


def polygon_nodes(verts, p):
    """p nodes equispaced by arc length (midpoint offset) along a closed polygon."""
    v = np.asarray(verts, dtype=np.float64)
    seg = np.roll(v, -1, axis=0) - v
    L = np.linalg.norm(seg, axis=1)
    cum = np.concatenate([[0.0], np.cumsum(L)])
    s = (np.arange(p) + 0.5) * cum[-1] / p
    e = np.searchsorted(cum, s, side="right") - 1
    t = (s - cum[e]) / L[e]
    return v[e] + t[:, None] * seg[e]


def cube_face_nodes(per_side, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    t = (np.arange(per_side) + 0.5) / per_side
    a, b = np.meshgrid(t, t, indexing="ij")
    a = a.ravel()
    b = b.ravel()
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    faces = []
    for ax in range(3):
        o = [q for q in range(3) if q != ax]
        for side in (lo[ax], hi[ax]):
            pts = np.empty((len(a), 3))
            pts[:, ax] = side
            pts[:, o[0]] = lo[o[0]] + (hi[o[0]] - lo[o[0]]) * a
            pts[:, o[1]] = lo[o[1]] + (hi[o[1]] - lo[o[1]]) * b
            faces.append(pts)
    return np.concatenate(faces)


# --------------------------------------------------- the paper's layouts


def paper_disk_layout():
    """Rings r_k = (k - 1/2)/10, 6k - 3 equispaced points each, k = 1..10
    (n = 300), and 60 boundary nodes."""
    pts = []
    for k in range(1, 11):
        nk = 6 * k - 3
        r = (k - 0.5) / 10.0
        th = 2.0 * np.pi * np.arange(nk) / nk
        pts.append(np.stack([r * np.cos(th), r * np.sin(th)], axis=1))
    return np.concatenate(pts), circle_nodes(60)


def plaplace_torsion_disk_exact(x, P):
    """Exact solution of the paper's p-torsion example on the unit disk
    (-div(|grad u|^(P-2) grad u) = 1, u = 0 on the circle):
    (P-1)/P (1/2)^(1/(P-1)) (1 - |x|^(P/(P-1))).  Problem data for
    reporting errors, like the manufactured solutions here."""
    r2 = np.sum(np.asarray(x, dtype=np.float64) ** 2, axis=-1)
    return (P - 1.0) / P * 0.5 ** (1.0 / (P - 1.0)) * (1.0 - np.power(r2, P / (2.0 * P - 2.0)))


def elliptic_divmin_disk(x):
    """The example "elliptic div min" on the unit disk: A = [[1, xy], [xy, 1]],
    phi = (x^2 + y^2) / 2, c = 1, u = (1 - x^2 - y^2)(x^3 - 3 x y^2) (0 on
    the circle).  Returns u, grad u (n, 2) and f = -div(A grad u) +
    (A grad phi).grad u + c u, by hand-differentiated closed forms.  Problem
    data, like the manufactured solutions here."""
    x = np.asarray(x, dtype=np.float64)
    X, Y = x[:, 0], x[:, 1]
    s = 1.0 - X * X - Y * Y
    h = X ** 3 - 3 * X * Y * Y
    hx, hy = 3 * X * X - 3 * Y * Y, -6 * X * Y
    hxx, hxy, hyy = 6 * X, -6 * Y, -6 * X
    sx, sy = -2 * X, -2 * Y
    u = s * h
    ux, uy = s * hx + h * sx, s * hy + h * sy
    uxx = -2 * h + 2 * sx * hx + s * hxx
    uyy = -2 * h + 2 * sy * hy + s * hyy
    uxy = sx * hy + sy * hx + s * hxy
    div = uxx + uyy + 2 * X * Y * uxy + X * ux + Y * uy  # div(A grad u)
    agx, agy = X + X * Y * Y, X * X * Y + Y            # A grad phi
    f = -div + agx * ux + agy * uy + u
    return u, np.stack([ux, uy], 1), f


def elliptic_div_disk(x):
    """The example "elliptic div" on the unit disk: div(A grad u) + b.grad u
    - c u = f with A = [[2 + x^2, xy], [xy, 2 + y^2]], b = (-y, x), c = 1 and
    u = (1 - x^2 - y^2) sin(pi x) (0 on the circle).  Returns u, grad u
    (n, 2) and f by hand-differentiated closed forms (div A = (3x, 3y)).
    Problem data, like the manufactured solutions here."""
    x = np.asarray(x, dtype=np.float64)
    X, Y = x[:, 0], x[:, 1]
    s = 1.0 - X * X - Y * Y
    sn, cs = np.sin(np.pi * X), np.cos(np.pi * X)
    u = s * sn
    ux = -2 * X * sn + s * np.pi * cs
    uy = -2 * Y * sn
    uxx = -2 * sn - 4 * X * np.pi * cs - s * np.pi ** 2 * sn
    uyy = -2 * sn
    uxy = -2 * Y * np.pi * cs
    div = (2 + X * X) * uxx + 2 * X * Y * uxy + (2 + Y * Y) * uyy + 3 * X * ux + 3 * Y * uy
    f = div + (-Y) * ux + X * uy - u
    return u, np.stack([ux, uy], 1), f


def elliptic_div_coef(x):
    """The example's coefficients at the sites: A (n, 2, 2), b (n, 2), c (n,)."""
    x = np.asarray(x, dtype=np.float64)
    X, Y = x[:, 0], x[:, 1]
    A = np.stack([np.stack([2 + X * X, X * Y], -1), np.stack([X * Y, 2 + Y * Y], -1)], -2)
    return A, np.stack([-Y, X], 1), np.ones(len(x))


def voronoi_l2_error(dom, sites, values, u_fn, npoints=1 << 21, seed=5):
    """Absolute L^2(D) distance between a function u_fn (callable on points
    (k, d)) and the piecewise-constant field equal to values[i] on the
    Voronoi cell of sites[i]: (sum_i int_{V_i} (u - values_i)^2)^(1/2), by
    Monte Carlo over uniform points of the domain's bounding box (the
    measure of Table "errors" of the examples)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    lo, hi = bbox(dom)
    tree = cKDTree(np.asarray(sites, dtype=np.float64))
    values = np.asarray(values, dtype=np.float64)
    vol = float(np.prod(hi - lo))
    acc, chunk, done = 0.0, 1 << 18, 0
    while done < npoints:
        k = min(chunk, npoints - done)
        q = lo + (hi - lo) * rng.random((k, len(lo)))
        q = q[interior_with_margin(dom, q, 0.0)]
        if len(q):
            j = tree.query(q)[1]
            acc += float(((u_fn(q) - values[j]) ** 2).sum())
        done += k
    return np.sqrt(acc * vol / npoints)


def elliptic_divmin_coef(x):
    """The example's coefficient fields at the sites: A (n, 2, 2), c (n,)
    and the weight w = exp(-phi) (n,)."""
    x = np.asarray(x, dtype=np.float64)
    xy = x[:, 0] * x[:, 1]
    A = np.stack([np.stack([np.ones_like(xy), xy], -1), np.stack([xy, np.ones_like(xy)], -1)], -2)
    return A, np.ones(len(x)), np.exp(-0.5 * np.sum(x * x, axis=1))


def paper_square_layout():
    """20 x 20 cell centres of the unit square, 20 boundary nodes per edge."""
    g = (np.arange(20) + 0.5) / 20.0
    sites = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2)
    return sites, square_nodes(20)


# ------------------------------------------------------- configurations


def config(name, seed=20260807):
    """The benchmark configurations (sizes and seeds); returns a dict with
    domain, sites, bnodes, walks, eps, precision and a label."""
    if name == "disk64":
        dom = unit_disk()
        eps = 1e-3
        sites = sample_sites(dom, 64, seed, 10 * eps)
        return dict(name=name, domain=dom, sites=sites, bnodes=circle_nodes(64), walks=2000,
                    eps=eps, precision="f64", seed=seed,
                    label="2D unit disk, 64 sites, 64 boundary nodes, 2000 walks/site, eps 1e-3, FP64")
    if name == "square1024":
        dom = unit_square()
        eps = 1e-4
        sites = sample_sites(dom, 1024, seed, 10 * eps)
        return dict(name=name, domain=dom, sites=sites, bnodes=square_nodes(64), walks=10000,
                    eps=eps, precision="f32", seed=seed,
                    label="2D unit square, 1024 sites, 256 boundary nodes, 1e4 walks/site, eps 1e-4, FP32")
    if name == "ball4096":
        dom = unit_ball()
        eps = 1e-4
        sites = sample_sites(dom, 4096, seed, 10 * eps)
        return dict(name=name, domain=dom, sites=sites, bnodes=fibonacci_sphere(1024), walks=10000,
                    eps=eps, precision="f32", seed=seed,
                    label="3D unit ball, 4096 sites, 1024 Fibonacci boundary nodes, 1e4 walks/site, eps 1e-4")
    if name.startswith("lshape"):
        n = int(name[len("lshape"):])
        dom = l_shape()
        eps = 1e-4
        sites = sample_sites(dom, n, seed, 10 * eps)
        return dict(name=name, domain=dom, sites=sites, bnodes=polygon_nodes(dom["verts"], n // 4),
                    walks=10000, eps=eps, precision="f32", seed=seed,
                    label=f"2D L-shape, {n} sites, {n // 4} boundary nodes, 1e4 walks/site, eps 1e-4")
    if name == "cubeball32768":
        dom = cube_minus_ball()
        eps = 1e-5
        sites = sample_sites(dom, 32768, seed, 10 * eps)
        bn = np.concatenate([cube_face_nodes(34), fibonacci_sphere(1256, dom["center"], dom["radius"])])
        return dict(name=name, domain=dom, sites=sites, bnodes=bn, walks=100000, eps=eps,
                    precision="f32", seed=seed,
                    label="3D unit cube minus ball r=0.3, 32768 sites, 8192 boundary nodes, 1e5 walks/site, eps 1e-5")
    raise KeyError(name)


# ------------------------------------------- manufactured problem data


def smooth_field(seed, dim, terms=8, max_freq=3.0, scale=0.5):
    """A seeded smooth function sum_k a_k cos(w_k . x + phi_k) with its
    gradient and Laplacian in closed form.  Returns (f, grad, lap)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.normal(0.0, scale, terms)
    w = rng.normal(0.0, 1.0, (terms, dim))
    w *= (max_freq * rng.random(terms) ** (1.0 / dim) / np.linalg.norm(w, axis=1))[:, None]
    ph = rng.uniform(0, 2 * np.pi, terms)

    def val(x):
        x = np.atleast_2d(x)
        return np.cos(x @ w.T + ph) @ a

    def grad(x):
        x = np.atleast_2d(x)
        return -(np.sin(x @ w.T + ph) * a) @ w

    def lap(x):
        x = np.atleast_2d(x)
        return -np.cos(x @ w.T + ph) @ (a * (w * w).sum(axis=1))

    return val, grad, lap


# ------------------------------------------------ served request problems


def anisotropic_problem(seed, sites, bnodes, h=1e-5):
    """Data of one served request, -div(A grad u) + b . grad u = f with
    u = g on the boundary, on a 2-D domain (a manufactured solution):
    A(x) = R(t(x)) diag(1, k(x)) R(t(x))^T with k = 1 + 99 s(x), s in [0, 1]
    (anisotropy up to 1:100), b(x) = 0.8 (cos p(x), sin p(x)), and u_ex a
    seeded sum of cosines; t, s and p are smooth seeded fields.  f is derived
    from u_ex by central differences of the flux A grad u_ex (step h).
    Returns dict(A (n,2,2), b (n,2), f (n,), g (p,), u (n,) = u_ex at the
    sites)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    uex, ugrad, _ = smooth_field(int(rng.integers(1 << 30)), 2, terms=6, max_freq=2.5, scale=0.5)
    wt, wk, wp = (rng.normal(0.0, 1.5, 2) for _ in range(3))
    pt, pk, pp = rng.uniform(0, 2 * np.pi, 3)

    def coef(x):
        x = np.atleast_2d(x)
        t = np.pi * np.sin(x @ wt + pt)
        k = 1.0 + 99.0 * (0.5 + 0.5 * np.sin(x @ wk + pk))
        c, sn = np.cos(t), np.sin(t)
        R = np.stack([np.stack([c, -sn], -1), np.stack([sn, c], -1)], -2)
        D = np.zeros(R.shape)
        D[:, 0, 0] = 1.0
        D[:, 1, 1] = k
        A = R @ D @ np.transpose(R, (0, 2, 1))
        ph = x @ wp + pp
        b = 0.8 * np.stack([np.cos(ph), np.sin(ph)], 1)
        return A, b

    def flux(x):
        A, _ = coef(x)
        return np.einsum("nab,nb->na", A, ugrad(x))

    x = np.atleast_2d(np.asarray(sites, dtype=np.float64))
    A, b = coef(x)
    div = np.zeros(len(x))
    for a in range(2):
        e = np.zeros(2)
        e[a] = h
        div += (flux(x + e)[:, a] - flux(x - e)[:, a]) / (2.0 * h)
    f = -div + np.einsum("na,na->n", b, ugrad(x))
    return dict(A=A, b=b, f=f, g=uex(bnodes), u=uex(x))
