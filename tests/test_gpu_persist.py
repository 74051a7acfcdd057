"""Saved and loaded toolboxes (wos_toolbox_save / wos_toolbox_load): every
array, the statistics, and the solves of the loaded toolbox are the same
bits as the saved one's."""
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2608_07017_amd")

KEYS = ("A", "B", "H", "K", "Hcount", "lambda", "vcount", "lambda_v", "site_steps")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("case", ["square_f32", "cubeball_window", "disk_f64_wv"])
def test_save_load_round_trip(tmp_path, case):
    if case == "square_f32":
        dom = W.unit_square()
        sites = W.sample_sites(dom, 150, 3, 1e-3)
        kw = dict(bnodes=W.square_nodes(12), precision="f32")
    elif case == "cubeball_window":
        dom = W.cube_minus_ball()
        sites = W.sample_sites(dom, 200, 4, 1e-3)
        kw = dict(bnodes=np.concatenate([W.cube_face_nodes(3), W.fibonacci_sphere(30, dom["center"], dom["radius"])]),
                  precision="f32", tally="window", window_pages=2, window_bpages=1)
        rng0 = np.random.default_rng(2)
        kw.update(test_phi=rng0.normal(size=200), test_psi=rng0.normal(size=len(kw["bnodes"])))
    else:
        dom = W.unit_disk()
        sites = W.sample_sites(dom, 90, 5, 1e-3)
        kw = dict(bnodes=W.circle_nodes(24), precision="f64", vcentres=W.sample_sites(dom, 40, 6, 1e-3))
    bn = kw.pop("bnodes")
    _say("build", case)
    tb = P.Toolbox(dom, sites, bn, 700, 1e-4, seed=9, volume_samples=1 << 14, **kw)
    tb.build()
    torch.cuda.synchronize()
    path = tmp_path / ("%s.wostbx" % case)
    tb.save(path)
    t2 = P.Toolbox.load(path)
    i1, i2 = tb.info(), t2.info()
    for k in ("dim", "n", "m", "p", "precision", "walks_per_site", "walk_steps", "walks", "capped_walks",
              "max_walk_steps", "volume_inside"):
        assert i1[k] == i2[k], k
    keys = KEYS + (("moments",) if case == "cubeball_window" else ())
    for k in keys:
        assert torch.equal(tb.export(k), t2.export(k)), k
    # a solve on each gives the same bits
    n, p = tb.n, tb.p
    rng = np.random.default_rng(1)
    f, g = rng.normal(size=n), rng.normal(size=p)
    if tb.n == tb.m:
        u1, g1, _, _ = tb.solve(f, g, kind="linear", rcond=1e-2, solver="tikhonov")
        u2, g2, _, _ = t2.solve(f, g, kind="linear", rcond=1e-2, solver="tikhonov")
    else:
        fb = torch.tensor(rng.normal(size=tb.m), device="cuda")
        u1, g1 = tb.apply(fb, torch.tensor(g, device="cuda"))
        u2, g2 = t2.apply(fb, torch.tensor(g, device="cuda"))
    torch.cuda.synchronize()
    assert torch.equal(u1, u2) and torch.equal(g1, g2)
    # a rebuild of the loaded toolbox with the saved seed reproduces the build
    t2.build(seed=9)
    torch.cuda.synchronize()
    # (the fixed-point LDS sums of an FP32 toolbox do not depend on the order
    # of their additions; FP64 LDS sums and FP32 device atomics do, in their
    # last bits)
    assert torch.equal(tb.export("site_steps"), t2.export("site_steps"))
    if case == "square_f32":
        for k in ("A", "B", "Hcount", "K"):
            assert torch.equal(tb.export(k), t2.export(k)), k
    elif case == "disk_f64_wv":
        assert torch.equal(tb.export("Hcount"), t2.export("Hcount"))
        for k in ("A", "B", "K"):
            assert torch.allclose(tb.export(k), t2.export(k), rtol=1e-12, atol=1e-15), k
    else:
        assert torch.equal(tb.export("Hcount").sum(1), t2.export("Hcount").sum(1))
        # the loaded toolbox kept its test functions: the moments are rebuilt
        # (FP64 device atomics: equal up to the order of the additions)
        assert torch.allclose(tb.export("moments"), t2.export("moments"), rtol=1e-9, atol=1e-9)
    tb.free()
    t2.free()
