"""Cell weights lambda_i = |W_i| / |D| (oracle).

The weights of the cell-centre quadrature (Rem. "discretization" and the
definition of lambda_i in Sec. "Second order linear elliptic PDEs").  The
paper does not say how |W_i| is obtained; here it is estimated by uniform
points: Philox tag 1, counter (q mod 2^32, q >> 32, 0, 1) for block q; in
d = 2 a block gives two points (u0, u1), (u2, u3), in d = 3 one point
(u0, u1, u2); each coordinate is lo + (hi - lo) * u over the domain's
bounding box (one rounding per operation, no fused multiply-add).  Points
outside D are rejected; the rest are binned by nearest site, and
lambda_i = count_i / sum(count).  The counts are integers, and the GPU path
is asked to reproduce them exactly.

Pinned by tests/test_oracle_volume.py: sum(lambda) = 1, the exact volumes of
a regular layout on the unit square (lambda_i = 1/400 for the 20 x 20 cell
centres), and the disk's cell areas against their polygon areas.
"""
import numpy as np

from .geometry import inside, bounding_box
from .philox import philox4x32_10, to_uniform, seed_key, TAG_VOLUME
from .voronoi import nearest


def volume_points(dom, seed, npoints):
    """The first `npoints` candidate points of the volume stream (before rejection)."""
    return _points_range(dom, seed, 0, npoints)


def cell_counts(dom, sites, seed, npoints, chunk=1 << 20):
    sites = np.asarray(sites, dtype=np.float64)
    counts = np.zeros(len(sites), dtype=np.int64)
    d = dom["dim"]
    per = 2 if d == 2 else 1
    step = chunk - chunk % per
    for s in range(0, npoints, step):
        cnt = min(step, npoints - s)
        pts = _points_range(dom, seed, s, cnt)
        pts = pts[inside(dom, pts)]
        counts += np.bincount(nearest(sites, pts), minlength=len(sites))
    return counts


def _points_range(dom, seed, start, count):
    d = dom["dim"]
    per = 2 if d == 2 else 1
    b0 = start // per
    nblk = (count + per - 1) // per
    q = np.arange(b0, b0 + nblk, dtype=np.uint64)
    k0, k1 = seed_key(seed)
    w = philox4x32_10(q & np.uint64(0xFFFFFFFF), q >> np.uint64(32), 0, TAG_VOLUME, k0, k1)
    u = [to_uniform(x) for x in w]
    if d == 2:
        pts = np.stack([np.stack([u[0], u[1]], axis=1), np.stack([u[2], u[3]], axis=1)], axis=1)
        pts = pts.reshape(-1, 2)
    else:
        pts = np.stack([u[0], u[1], u[2]], axis=1)
    pts = pts[: count]
    lo, hi = bounding_box(dom)
    ext = hi - lo
    return lo + ext * pts


def cell_weights(dom, sites, seed, npoints):
    counts = cell_counts(dom, sites, seed, npoints)
    return counts / counts.sum(), counts
