"""Per-site moments of the four test functionals (GPU against the oracle).

With test values phi (one per V cell) and psi (one per boundary cell) the
build also sums, per site, each walk's value c of the estimators of
U phi, grad U phi, H psi and grad H psi, and its square (Sec. "Monte Carlo
estimators", eqs. u MC, gradu U MC, H MC, dh MC): the standard errors of the
binned toolbox applied to phi / psi follow from them.  The oracle computes
the same per-walk values from its own walks (oracle.walker.site_functionals).
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle.walker import site_functionals

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2608_07017_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy()


def _ref_moments(dom, sites, vc, bn, walks, eps, seed, phi, psi, rows):
    d = dom["dim"]
    out = np.zeros((len(rows), 4 + 4 * d))
    for r, i in enumerate(rows):
        cA, cB, cH, cK = site_functionals(dom, sites[i], int(i), walks, eps, seed, vc, bn, phi, psi)
        out[r, 0], out[r, 1] = cA.sum(), (cA * cA).sum()
        out[r, 2:2 + d], out[r, 2 + d:2 + 2 * d] = cB.sum(0), (cB * cB).sum(0)
        out[r, 2 + 2 * d], out[r, 3 + 2 * d] = cH.sum(), (cH * cH).sum()
        out[r, 4 + 2 * d:4 + 3 * d], out[r, 4 + 3 * d:] = cK.sum(0), (cK * cK).sum(0)
    return out


def _se(mom, N, d):
    """Standard errors of the four means from the sums (the header's formula)."""
    sums = np.concatenate([mom[:, 0:1], mom[:, 2:2 + d], mom[:, 2 + 2 * d:3 + 2 * d], mom[:, 4 + 2 * d:4 + 3 * d]], 1)
    sq = np.concatenate([mom[:, 1:2], mom[:, 2 + d:2 + 2 * d], mom[:, 3 + 2 * d:4 + 2 * d], mom[:, 4 + 3 * d:]], 1)
    mu = sums / N
    return mu, np.sqrt(np.maximum(sq / N - mu * mu, 0.0) / (N - 1))


@pytest.mark.parametrize("case", ["disk", "lshape_wv", "cubeball"])
def test_moments_fp64_match_oracle(case):
    """FP64: every walk is the oracle's, so the sums agree to rounding."""
    rng = np.random.default_rng(3)
    if case == "disk":
        dom, sites, bn, vc = W.unit_disk(), W.sample_sites(W.unit_disk(), 40, 5, 1e-3), W.circle_nodes(24), None
    elif case == "lshape_wv":
        dom = W.l_shape()
        sites = W.sample_sites(dom, 37, 6, 1e-3)
        vc = W.sample_sites(dom, 61, 7, 1e-3)
        bn = W.polygon_nodes(dom["verts"], 50)
    else:
        dom = W.cube_minus_ball()
        sites = W.sample_sites(dom, 29, 8, 1e-3)
        vc = None
        bn = np.concatenate([W.cube_face_nodes(3), W.fibonacci_sphere(30, dom["center"], dom["radius"])])
    d = dom["dim"]
    m = len(sites) if vc is None else len(vc)
    phi, psi = rng.normal(size=m), rng.normal(size=len(bn))
    walks, eps, seed = 700, 1e-3, 19
    _say("GPU moments FP64:", case, "n=%d m=%d p=%d" % (len(sites), m, len(bn)))
    tb = P.Toolbox(dom, sites, bn, walks, eps, seed=seed, precision="f64", volume_samples=1 << 12, vcentres=vc,
                   test_phi=phi, test_psi=psi)
    tb.build()
    torch.cuda.synchronize()
    got = _np(tb.export("moments"))
    assert got.shape == (len(sites), 4 + 4 * d)
    ref = _ref_moments(dom, sites, sites if vc is None else vc, bn, walks, eps, seed, phi, psi,
                       np.arange(len(sites)))
    scale = np.abs(ref).max(axis=0, keepdims=True)
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-11 * scale)
    # the means are the toolbox applied to phi / psi
    A, B, H, K = (_np(tb.export(k)) for k in ("A", "B", "H", "K"))
    mu, _ = _se(got, walks, d)
    assert np.allclose(mu[:, 0], A @ phi, rtol=1e-10, atol=1e-12)
    assert np.allclose(mu[:, 1:1 + d], (B @ phi).T, rtol=1e-10, atol=1e-11)
    assert np.allclose(mu[:, 1 + d], H @ psi, rtol=1e-10, atol=1e-12)
    assert np.allclose(mu[:, 2 + d:], (K @ psi).T, rtol=1e-10, atol=1e-11)
    # a second build starts the sums from zero again
    tb.build()
    torch.cuda.synchronize()
    assert np.allclose(_np(tb.export("moments")), got, rtol=1e-12, atol=1e-13 * scale)


def test_moments_fp32_window_mode_cube_minus_ball():
    """FP32 in the windowed tally mode (test values permuted with the
    columns) against the LDS-row mode on the same walks and against the
    oracle on sampled rows: the means within 4 standard errors (the FP32
    walks are the oracle's up to rounding) and the standard errors within
    10 %."""
    dom = W.cube_minus_ball()
    sites = W.sample_sites(dom, 333, 23, 1e-3)
    bn = np.concatenate([W.cube_face_nodes(4), W.fibonacci_sphere(54, dom["center"], dom["radius"])])
    rng = np.random.default_rng(4)
    phi, psi = rng.normal(size=len(sites)), rng.normal(size=len(bn))
    walks, eps, seed = 2000, 1e-4, 13
    kw = dict(precision="f32", volume_samples=1 << 12, test_phi=phi, test_psi=psi)
    _say("GPU moments FP32: lds_rows and window")
    t1 = P.Toolbox(dom, sites, bn, walks, eps, seed=seed, **kw).build()
    t2 = P.Toolbox(dom, sites, bn, walks, eps, seed=seed, tally="window", window_pages=2, window_bpages=1,
                   **kw).build()
    torch.cuda.synchronize()
    m1, m2 = _np(t1.export("moments")), _np(t2.export("moments"))
    d = 3
    mu1, se1 = _se(m1, walks, d)
    mu2, se2 = _se(m2, walks, d)
    # the same walks: equal up to FP32 rounding and the odd exact tie
    assert np.all(np.abs(mu1 - mu2) <= 1e-4 * np.abs(mu1).max(0) + 0.2 * se1)
    assert np.allclose(se1, se2, rtol=2e-2, atol=1e-6)
    # the means are the toolbox applied to phi / psi
    A, H = _np(t1.export("A")).astype(np.float64), _np(t1.export("H")).astype(np.float64)
    assert np.allclose(mu1[:, 0], A @ phi, rtol=0, atol=1e-4 * (np.abs(A) @ np.abs(phi)).max())
    assert np.allclose(mu1[:, 1 + d], H @ psi, rtol=0, atol=1e-4 * np.abs(psi).max())
    rows = np.array([0, 57, 190, 332])
    ref = _ref_moments(dom, sites, sites, bn, walks, eps, seed, phi, psi, rows)
    mur, ser = _se(ref, walks, d)
    assert np.all(np.abs(mu2[rows] - mur) <= 4 * ser + 1e-6)
    assert np.allclose(se2[rows], ser, rtol=0.1, atol=1e-6)


def test_moments_need_both_test_functions():
    dom = W.unit_disk()
    sites = W.sample_sites(dom, 10, 5, 1e-3)
    with pytest.raises(ValueError):
        P.Toolbox(dom, sites, W.circle_nodes(8), 10, 1e-3, test_phi=np.ones(10))
    with pytest.raises(ValueError):
        P.Toolbox(dom, sites, W.circle_nodes(8), 10, 1e-3, test_phi=np.ones(9), test_psi=np.ones(8))
