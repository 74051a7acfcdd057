"""Domains, the distance to the boundary r(x) and inside tests (oracle).

r(x) = inf_{y on the boundary} |x - y|, eq. (r) of Sec. "Probabilistic
representations"; it is the radius of every Walk-on-Spheres step (eq. wos
chain).  Domains supported (the ones the workloads use):

* ``ball``            -- disk (d=2) or ball (d=3): centre c, radius R;
* ``box``             -- axis-aligned box [lo, hi];
* ``polygon``         -- simple polygon (d=2), vertices counter-clockwise;
* ``box_minus_ball``  -- box [lo, hi] with the closed ball |x-c| <= R removed.

A domain is a plain dict: {"kind", "dim", "center", "radius", "lo", "hi",
"verts"} (unused keys may be absent).

Pinned by tests/test_oracle_geometry.py: closed forms for ball/box, brute
force over densely sampled boundary points for the polygon and the
box-minus-ball, and the crossing-number test against points known to be
inside/outside the L-shape.
"""
import numpy as np


def _arr(x):
    return np.atleast_2d(np.asarray(x, dtype=np.float64))


def _sq_norm(v):
    """Squared norm summed left to right: ((v0^2 + v1^2) + v2^2)."""
    acc = v[:, 0] * v[:, 0]
    for a in range(1, v.shape[1]):
        acc = acc + v[:, a] * v[:, a]
    return acc


def _box_dist(x, lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return np.minimum(x - lo, hi - x).min(axis=1)


def _seg_dist(x, a, b):
    """Distance from points x (k,2) to the segment [a, b]."""
    ab = b - a
    t = ((x - a) @ ab) / (ab @ ab)
    t = np.clip(t, 0.0, 1.0)
    proj = a + t[:, None] * ab
    return np.linalg.norm(x - proj, axis=1)


def distance(dom, x):
    """r(x) for points x (k, d); valid for x in the closure of D."""
    x = _arr(x)
    kind = dom["kind"]
    if kind == "ball":
        c = np.asarray(dom["center"], dtype=np.float64)
        return dom["radius"] - np.linalg.norm(x - c, axis=1)
    if kind == "box":
        return _box_dist(x, dom["lo"], dom["hi"])
    if kind == "polygon":
        v = np.asarray(dom["verts"], dtype=np.float64)
        nv = len(v)
        d = np.full(len(x), np.inf)
        for e in range(nv):
            d = np.minimum(d, _seg_dist(x, v[e], v[(e + 1) % nv]))
        return d
    if kind == "box_minus_ball":
        c = np.asarray(dom["center"], dtype=np.float64)
        return np.minimum(_box_dist(x, dom["lo"], dom["hi"]),
                          np.linalg.norm(x - c, axis=1) - dom["radius"])
    raise ValueError(kind)


def inside(dom, x):
    """Interior test.  Balls compare squared norms (no square root); the
    polygon uses the even-odd crossing rule (points exactly on an edge are
    not resolved; the volume points never land on the lattice lines of the
    workloads' polygons)."""
    x = _arr(x)
    kind = dom["kind"]
    if kind == "ball":
        c = np.asarray(dom["center"], dtype=np.float64)
        return _sq_norm(x - c) < dom["radius"] * dom["radius"]
    if kind == "box":
        return np.all((x > np.asarray(dom["lo"])) & (x < np.asarray(dom["hi"])), axis=1)
    if kind == "polygon":
        v = np.asarray(dom["verts"], dtype=np.float64)
        nv = len(v)
        odd = np.zeros(len(x), dtype=bool)
        for e in range(nv):
            a, b = v[e], v[(e + 1) % nv]
            crosses = (a[1] > x[:, 1]) != (b[1] > x[:, 1])
            with np.errstate(divide="ignore", invalid="ignore"):
                xint = a[0] + (x[:, 1] - a[1]) * (b[0] - a[0]) / (b[1] - a[1])
            odd ^= crosses & (x[:, 0] < xint)
        return odd
    if kind == "box_minus_ball":
        c = np.asarray(dom["center"], dtype=np.float64)
        inbox = np.all((x > np.asarray(dom["lo"])) & (x < np.asarray(dom["hi"])), axis=1)
        return inbox & (_sq_norm(x - c) > dom["radius"] * dom["radius"])
    raise ValueError(kind)


def bounding_box(dom):
    kind = dom["kind"]
    d = dom["dim"]
    if kind == "ball":
        c = np.asarray(dom["center"], dtype=np.float64)[:d]
        return c - dom["radius"], c + dom["radius"]
    if kind in ("box", "box_minus_ball"):
        return (np.asarray(dom["lo"], dtype=np.float64)[:d],
                np.asarray(dom["hi"], dtype=np.float64)[:d])
    if kind == "polygon":
        v = np.asarray(dom["verts"], dtype=np.float64)
        return v.min(axis=0), v.max(axis=0)
    raise ValueError(kind)
