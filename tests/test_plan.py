"""Host decisions of a build (wos_toolbox_plan): tally mode, accumulators,
work split, windows, and the fixed-point overflow guard.  Host only: no
device call is made."""
import numpy as np
import pytest

import workloads as W
import paper_2608_07017_amd as P


def _plan(name, **kw):
    c = W.config(name)
    kw.setdefault("precision", c["precision"])
    return P.build_plan(c["domain"], c["sites"], c["bnodes"], c["walks"], c["eps"], **kw)


def test_workload_plans():
    # rows in LDS while they fit, the windowed mode for the 32768-site box
    # minus ball (its rows take 640 KB), one walker workgroup per compute unit,
    # fixed-point sums
    assert _plan("square1024")["tally_mode"] == "lds_rows"
    assert _plan("ball4096")["tally_mode"] == "lds_rows"
    cb = _plan("cubeball32768")
    assert cb["tally_mode"] == "window"
    assert cb["window_bpages"] == 8 and 40 <= cb["window_pages"] <= 255
    assert 140 * 1024 <= cb["lds_bytes"] <= 160 * 1024
    assert cb["tally_acc"] == "fixed" and cb["fixed_bound"] < 0.5
    assert cb["items_per_site"] * cb["walks_per_item"] >= 100000


def test_window_size_options():
    pl = _plan("cubeball32768", window_pages=50, window_bpages=24)
    assert pl["window_pages"] == 50 and pl["window_bpages"] == 24
    # 8 (1 + d) 64 bytes per V page, (8 d + 4) 64 per boundary page, plus
    # tables and lists
    assert pl["lds_bytes"] == 8 * 4 * 64 * 50 + 28 * 64 * 24 + 2 * 74 + 512 + 128
    with pytest.raises(P.WosError):   # more than LDS holds
        _plan("cubeball32768", window_pages=255, window_bpages=255)


def test_forced_modes_and_their_limits():
    assert _plan("square1024", tally="window")["tally_mode"] == "window"
    assert _plan("square1024", tally="hbm")["tally_mode"] == "hbm"
    with pytest.raises(P.WosError):
        _plan("cubeball32768", tally="lds_rows")
    with pytest.raises(P.WosError):
        _plan("disk64", tally="window")          # FP64 toolbox
    with pytest.raises(P.WosError):
        _plan("square1024", walker_block=300)
    with pytest.raises(P.WosError):
        _plan("cubeball32768", tally="window", tally_acc="f64")   # the window sums in fixed point


def _near_boundary_case(r0, walks, **kw):
    dom = W.unit_square()
    sites = np.array([[0.5, 0.5], [r0, 0.5]])
    return P.build_plan(dom, sites, W.square_nodes(4), walks, 1e-9, walks_per_item=walks, **kw)


def test_fixed_point_bound_formula():
    # K: N d / r0, B: 4 N (d / r0) R^2 / d, A: 4 N omega_max R^2 / d, with
    # R^2 = 1/2 (half diagonal of the unit square) and omega_max = 12 in 2-D
    N, r0 = 1000, 1e-3
    pl = _near_boundary_case(r0, N)
    bK = N * 2 / r0
    bB = 4 * N * (2 / r0) * 0.5 / 2
    bA = 4 * N * 12 * 0.5 / 2
    assert np.isclose(pl["fixed_bound"], max(bK, bB, bA) / 2 ** 31, rtol=1e-12)
    assert pl["tally_acc"] == "fixed"


def test_fixed_point_overflow_guard():
    # a site 1e-6 from the boundary with 1e5 walks in one item: a K sum can
    # reach 2e11 > 2^31, so the automatic choice is FP64 and forcing fixed
    # point is refused
    pl = _near_boundary_case(1e-6, 100000)
    assert pl["fixed_bound"] >= 0.5
    assert pl["tally_acc"] == "f64"
    assert _near_boundary_case(1e-6, 100000, tally_acc="f64")["tally_acc"] == "f64"
    with pytest.raises(P.WosError):
        _near_boundary_case(1e-6, 100000, tally_acc="fixed")
    # smaller items bring the bound back into range
    small = P.build_plan(W.unit_square(), np.array([[0.5, 0.5], [1e-6, 0.5]]), W.square_nodes(4), 100000, 1e-9,
                         walks_per_item=100)
    assert small["fixed_bound"] < 0.5 and small["tally_acc"] == "fixed"


def test_window_items_are_split_for_fixed_point():
    # the windowed mode always sums in fixed point: a site 1e-6 from the
    # boundary splits its 1e5 walks into items that keep the bound below 1/2
    # (per walk: 4 (d / r0) R^2 / d with R^2 = 1/2 -> 2e6; items of at most
    # 0.49 2^31 / 2e6 = 526 walks); automatic mode takes it as long as the
    # items keep at least 256 walks, else the HBM mode
    pl = _near_boundary_case(1e-6, 100000, tally="window")
    assert pl["tally_mode"] == "window" and pl["tally_acc"] == "fixed"
    assert pl["walks_per_item"] == int(0.49 * 2 ** 31 / 2e6)
    assert pl["fixed_bound"] < 0.5
    assert pl["items_per_site"] * pl["walks_per_item"] >= 100000
    with pytest.raises(P.WosError):
        _near_boundary_case(1e-10, 1000, tally="window")      # not even one walk per item fits
    dom = W.unit_square()
    sites = np.concatenate([W.sample_sites(dom, 8000, 3, 1e-3), [[1e-7, 0.5]]])
    auto = P.build_plan(dom, sites, W.square_nodes(4), 100000, 1e-9)
    assert auto["tally_mode"] == "hbm"          # rows beyond LDS, items of 52 walks would be too small


def test_window_items_follow_each_sites_own_bound():
    # in the windowed mode each site is split by its own bound: with 4000
    # walks, the site 1e-6 from the boundary takes items of 0.49 2^31 / 2e6
    # = 526 walks (8 items), the 40 sites at least 1e-3 from it larger ones;
    # the plan reports the smallest item, the most items of a site and the
    # largest bound
    dom = W.unit_square()
    sites = np.concatenate([W.sample_sites(dom, 40, 31, 1e-3), [[1e-6, 0.5]]])
    pl = P.build_plan(dom, sites, W.square_nodes(24), 4000, 1e-4, tally="window", window_pages=1, window_bpages=1)
    assert pl["walks_per_item"] == int(0.49 * 2 ** 31 / 2e6) and pl["items_per_site"] == 8
    assert 0.48 < pl["fixed_bound"] < 0.5
    # without the near site only the load balance splits the sites (items
    # of at least 4 walks per lane of a workgroup), far below their bounds
    pl2 = P.build_plan(dom, sites[:-1], W.square_nodes(24), 4000, 1e-4, tally="window", window_pages=1,
                       window_bpages=1)
    assert pl2["walks_per_item"] >= 1024 and pl2["items_per_site"] * pl2["walks_per_item"] >= 4000
    assert pl2["fixed_bound"] < 0.01


def test_plan_rejects_bad_inputs():
    dom = W.unit_disk()
    with pytest.raises(P.WosError):
        P.build_plan(dom, np.array([[2.0, 0.0]]), W.circle_nodes(8), 10, 1e-3)   # site outside
    with pytest.raises(P.WosError):
        P.build_plan(dom, np.array([[0.1, 0.0]]), W.circle_nodes(8), 10, 1e-3, window_pages=300)
