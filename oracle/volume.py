"""Cell weights lambda_i = |W_i| / |D| (oracle).

The weights of the cell-centre quadrature (Rem. "discretization" and the
definition of lambda_i in Sec. "Second order linear elliptic PDEs").  The
paper does not say how |W_i| is obtained; here it is estimated by
stratified uniform points over the domain's bounding box: the box is cut
into T^d equal tiles (T a power of two, the largest with at least 64
points per tile) and every tile receives K points, uniform within it, K
the largest power of two with K T^d <= npoints (K T^d candidate points in
all, at least half the requested number).  Point p lies in tile
p // K (tiles in row-major order, last axis fastest) and takes its
uniforms from Philox tag 1, counter (q mod 2^32, q >> 32, 0, 1) for block
q; in d = 2 a block gives two points (u0, u1), (u2, u3), in d = 3 one
point (u0, u1, u2).  Coordinate a is lo_a + (hi_a - lo_a) * ((c_a + u_a) / T)
with c_a the tile's index on that axis (one rounding per operation, no
fused multiply-add; c + u and the division by T are exact).  Points
outside D are rejected; the rest are binned by nearest site, and
lambda_i = count_i / sum(count), an unbiased estimate of the volume
fraction (stratification only lowers its variance).  The counts are
integers, and the GPU path is asked to reproduce them exactly.

Pinned by tests/test_oracle_volume.py: sum(lambda) = 1, the exact volumes of
a regular layout on the unit square (lambda_i = 1/400 for the 20 x 20 cell
centres), and the disk's cell areas against their polygon areas.
"""
import numpy as np

from .geometry import inside, bounding_box
from .philox import philox4x32_10, to_uniform, seed_key, TAG_VOLUME
from .voronoi import nearest


MIN_PER_TILE = 64


def volume_layout(dim, npoints):
    """(T, K): tiles per axis and points per tile for `npoints` requested
    points, both powers of two (K T^d <= npoints, at least half of it)."""
    T, K = 1, 1
    while (2 * T) ** dim * MIN_PER_TILE <= npoints:
        T *= 2
    while 2 * K * T ** dim <= npoints:
        K *= 2
    return T, K


def volume_points(dom, seed, npoints):
    """All K T^d candidate points of the volume stream (before rejection)."""
    T, K = volume_layout(dom["dim"], npoints)
    return _points_range(dom, seed, 0, K * T ** dom["dim"], T, K)


def cell_counts(dom, sites, seed, npoints, chunk=1 << 20):
    sites = np.asarray(sites, dtype=np.float64)
    counts = np.zeros(len(sites), dtype=np.int64)
    d = dom["dim"]
    T, K = volume_layout(d, npoints)
    total = K * T ** d
    per = 2 if d == 2 else 1
    step = chunk - chunk % per
    for s in range(0, total, step):
        cnt = min(step, total - s)
        pts = _points_range(dom, seed, s, cnt, T, K)
        pts = pts[inside(dom, pts)]
        counts += np.bincount(nearest(sites, pts), minlength=len(sites))
    return counts


def _points_range(dom, seed, start, count, T, K):
    d = dom["dim"]
    per = 2 if d == 2 else 1
    b0 = start // per
    nblk = (count + per - 1) // per
    q = np.arange(b0, b0 + nblk, dtype=np.uint64)
    k0, k1 = seed_key(seed)
    w = philox4x32_10(q & np.uint64(0xFFFFFFFF), q >> np.uint64(32), 0, TAG_VOLUME, k0, k1)
    u = [to_uniform(x) for x in w]
    if d == 2:
        uu = np.stack([np.stack([u[0], u[1]], axis=1), np.stack([u[2], u[3]], axis=1)], axis=1)
        uu = uu.reshape(-1, 2)
    else:
        uu = np.stack([u[0], u[1], u[2]], axis=1)
    p0 = b0 * per
    uu = uu[start - p0: start - p0 + count]
    # tile coordinates of each point (row-major tiles, last axis fastest)
    tile = np.arange(start, start + count, dtype=np.int64) // K
    c = np.empty((count, d), dtype=np.float64)
    for a in range(d - 1, -1, -1):
        c[:, a] = tile % T
        tile //= T
    frac = (c + uu) / T          # both steps exact
    lo, hi = bounding_box(dom)
    ext = hi - lo
    return lo + ext * frac


def cell_weights(dom, sites, seed, npoints):
    counts = cell_counts(dom, sites, seed, npoints)
    return counts / counts.sum(), counts
