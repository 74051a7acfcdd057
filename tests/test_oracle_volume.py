"""Pins of the cell weights lambda_i = |W_i|/|D|."""
import numpy as np

import workloads as W
from oracle.volume import cell_weights, cell_counts, volume_points, volume_layout
from oracle.geometry import inside


def _clip(poly, a, c):
    """Keep the part of polygon `poly` with a . x <= c (Sutherland-Hodgman)."""
    out = []
    n = len(poly)
    for k in range(n):
        P, Q = poly[k], poly[(k + 1) % n]
        fp, fq = a @ P - c, a @ Q - c
        if fp <= 0:
            out.append(P)
        if fp * fq < 0:
            t = fp / (fp - fq)
            out.append(P + t * (Q - P))
    return np.array(out)


def _area(poly):
    x, y = poly[:, 0], poly[:, 1]
    return 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))


def exact_box_voronoi_areas(sites):
    box = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    areas = []
    for i, s in enumerate(sites):
        poly = box
        for j, t in enumerate(sites):
            if j != i:
                a = t - s                      # keep |x-s| <= |x-t|
                c = 0.5 * (t @ t - s @ s)
                poly = _clip(poly, a, c)
        areas.append(_area(poly))
    return np.array(areas)


def test_counts_match_exact_voronoi_areas():
    sites = W.sample_sites(W.unit_square(), 40, 17, 0.0)
    exact = exact_box_voronoi_areas(sites)
    assert np.isclose(exact.sum(), 1.0)
    npts = 1 << 20
    lam, counts = cell_weights(W.unit_square(), sites, 77, npts)
    assert counts.sum() == npts                 # box: nothing rejected
    se = np.sqrt(exact * (1 - exact) / npts)
    assert np.all(np.abs(lam - exact) <= 5 * se)
    assert np.isclose(lam.sum(), 1.0)


def test_paper_square_layout_is_uniform():
    sites, _ = W.paper_square_layout()
    lam, counts = cell_weights(W.unit_square(), sites, 5, 1 << 20)
    se = np.sqrt(1 / 400 * (1 - 1 / 400) / (1 << 20))
    assert np.all(np.abs(lam - 1 / 400) <= 5 * se)


def test_disk_rejection_fraction():
    # fraction of bounding-box points kept is pi / 4
    npts = 1 << 20
    sites, _ = W.paper_disk_layout()
    counts = cell_counts(W.unit_disk(), sites, 3, npts)
    frac = counts.sum() / npts
    assert abs(frac - np.pi / 4) < 5 * np.sqrt(np.pi / 4 * (1 - np.pi / 4) / npts)
    # the rings layout has cells of about pi/300 (paper: lambda ~ 1e-2)
    lam = counts / counts.sum()
    assert 0.8 / 300 < lam.min() and lam.max() < 1.2 / 300


def test_point_stream_is_in_bbox_and_off_lattice():
    pts = volume_points(W.l_shape(), 9, 100001)
    T, K = volume_layout(2, 100001)
    assert (T, K) == (32, 64) and pts.shape == (K * T * T, 2)
    assert np.all(np.abs(pts) < 1)
    assert not np.any(pts == 0.0)
    kept = inside(W.l_shape(), pts).mean()
    assert abs(kept - 0.75) < 0.01


def test_points_are_stratified_by_tile():
    """Every tile of the bounding box receives exactly K points, uniform in
    it: tile counts are exact, and within-tile offsets have mean 1/2 and
    variance 1/12 (the uniform law's) to sampling precision."""
    for dom, n in ((W.unit_square(), 1 << 14), (W.unit_ball(), 1 << 15)):
        d = dom["dim"]
        T, K = volume_layout(d, n)
        assert K >= 64 and K * T ** d <= n < 2 * K * T ** d
        pts = volume_points(dom, 3, n)
        lo = -np.ones(d) if dom["kind"] == "ball" else np.zeros(d)
        ext = 2.0 * np.ones(d) if dom["kind"] == "ball" else np.ones(d)
        rel = (pts - lo) / ext * T
        cell = np.floor(rel).astype(np.int64)
        lin = np.ravel_multi_index(tuple(cell.T), (T,) * d)
        assert np.array_equal(np.bincount(lin, minlength=T ** d), np.full(T ** d, K))
        off = rel - cell
        assert np.allclose(off.mean(axis=0), 0.5, atol=5 / np.sqrt(12 * len(off)))
        assert np.allclose(off.var(axis=0), 1 / 12, atol=5 * np.sqrt(1 / 180 / len(off)))
        # consecutive points share a tile: the first K points are all in tile 0
        assert np.all(lin[:K] == 0) and np.all(lin[K:2 * K] == 1)
