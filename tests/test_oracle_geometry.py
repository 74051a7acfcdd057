"""Pins of r(x) (eq. r) and the inside tests."""
import numpy as np

import workloads as W
from oracle.geometry import distance, inside


def _brute_dist(boundary_pts, x):
    d2 = ((x[:, None, :] - boundary_pts[None]) ** 2).sum(axis=2)
    return np.sqrt(d2.min(axis=1))


def test_disk_and_ball_closed_form():
    x = np.array([[0.3, 0.4], [0.0, 0.0], [-0.9, 0.1]])
    assert np.allclose(distance(W.unit_disk(), x), 1 - np.linalg.norm(x, axis=1), atol=0, rtol=1e-15)
    x3 = np.array([[0.3, 0.4, 0.5], [0.0, 0.0, 0.0]])
    assert np.allclose(distance(W.unit_ball(), x3), 1 - np.linalg.norm(x3, axis=1))


def test_box_closed_form():
    x = np.array([[0.1, 0.5], [0.7, 0.95], [0.5, 0.5]])
    assert np.allclose(distance(W.unit_square(), x), [0.1, 0.05, 0.5])


def test_polygon_against_dense_boundary():
    dom = W.l_shape()
    bpts = W.polygon_nodes(dom["verts"], 80000)
    x = W.sample_sites(dom, 500, 3, 0.0)
    assert np.all(inside(dom, x))
    r = distance(dom, x)
    rb = _brute_dist(bpts, x)
    # the dense sampling is 1e-4 apart: brute force over-estimates by < 5e-5
    assert np.all(r <= rb + 1e-12) and np.all(rb - r < 6e-5)
    # the re-entrant corner: distance from (0.5,-0.5) is 0.5*sqrt(2)? no: it is
    # outside; from (0.3,0.1) the nearest boundary is the edge y=0, x in [0,1]
    assert np.isclose(distance(dom, np.array([[0.3, 0.1]]))[0], 0.1)
    assert np.isclose(distance(dom, np.array([[-0.1, -0.2]]))[0], 0.1)
    assert np.isclose(distance(dom, np.array([[0.3, 0.1]]))[0], 0.1)


def test_polygon_inside():
    dom = W.l_shape()
    inn = np.array([[-0.5, -0.5], [0.5, 0.5], [-0.5, 0.5], [-0.01, -0.99]])
    out = np.array([[0.5, -0.5], [1.5, 0.0], [0.01, -0.01], [-1.01, 0.0]])
    assert np.all(inside(dom, inn))
    assert not np.any(inside(dom, out))


def test_cube_minus_ball():
    dom = W.cube_minus_ball()
    x = W.sample_sites(dom, 300, 4, 0.0)
    assert np.all(inside(dom, x))
    k = 60
    g = (np.arange(k) + 0.5) / k
    a, b = np.meshgrid(g, g, indexing="ij")
    faces = W.cube_face_nodes(200)
    sph = W.fibonacci_sphere(40000, dom["center"], dom["radius"])
    rb = _brute_dist(np.concatenate([faces, sph]), x)
    r = distance(dom, x)
    assert np.all(np.abs(r - rb) < 6e-3)
    assert np.isclose(distance(dom, np.array([[0.5, 0.5, 0.85]]))[0], 0.05)
    assert not inside(dom, np.array([[0.5, 0.5, 0.6]]))[0]
