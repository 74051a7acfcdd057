"""Pins of the nearest-centre map (brute force, lowest index on ties)."""
import numpy as np

from oracle.voronoi import nearest


def test_lattice_known_cells():
    g = (np.arange(10) + 0.5) / 10
    sites = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2)
    rng = np.random.default_rng(0)
    q = rng.random((5000, 2))
    ix = np.minimum((q * 10).astype(int), 9)
    expect = ix[:, 0] * 10 + ix[:, 1]
    assert np.array_equal(nearest(sites, q), expect)


def test_ties_go_to_lowest_index():
    sites = np.array([[1.0, 0.0], [-1.0, 0.0], [0.0, 1.0], [0.0, -1.0]])
    assert nearest(sites, np.array([[0.0, 0.0]]))[0] == 0
    assert nearest(sites[::-1], np.array([[0.0, 0.0]]))[0] == 0
    assert nearest(sites[1:], np.array([[0.0, 0.0]]))[0] == 0
    assert nearest(sites, np.array([[0.0, 0.5]]))[0] == 2


def test_matches_scipy_kdtree_off_ties():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(3)
    sites = rng.random((700, 3))
    q = rng.random((20000, 3))
    _, j = cKDTree(sites).query(q)
    assert np.array_equal(nearest(sites, q), j)
