"""Host logic of the p-HiSD landscape search (paper_2608_07017_amd.search):
the dip finder, the square's symmetries as site permutations, and the
count of essentially distinct solutions.  No device call."""
import numpy as np
import pytest

import workloads as W
from paper_2608_07017_amd import search as S


def test_find_dip():
    # a transient dip (1e-4) that rises again 100-fold, then the final descent
    seq = [1.0, 0.1, 1e-2, 1e-4, 1e-3, 1e-2, 5e-3, 1e-5, 1e-7]
    assert S.find_dip(seq) == 3
    assert S.find_dip([1.0, 0.5, 0.1, 1e-3, 1e-6]) is None      # monotone: no dip
    assert S.find_dip([1.0, 1e-3, 2e-3, 1e-4]) is None          # the rise is below 10x
    assert S.find_dip([1.0, 1e-3, 2e-3, 1e-4], rise=1.5) == 1


def test_square_symmetries_form_the_dihedral_group():
    sites, _ = W.paper_square_layout()
    perms = S.square_symmetries(sites)
    assert len(perms) == 8
    assert len({tuple(p) for p in perms}) == 8
    assert np.array_equal(perms[0], np.arange(len(sites)))
    keys = {tuple(p) for p in perms}
    for a in perms:          # closed under composition, every element a permutation
        assert sorted(a) == list(range(len(sites)))
        for b in perms:
            assert tuple(a[b]) in keys
    with pytest.raises(ValueError):
        S.square_symmetries(sites + np.array([0.013, 0.0]))


def test_distinct_counts_symmetry_classes():
    sites, _ = W.paper_square_layout()
    perms = S.square_symmetries(sites)
    rng = np.random.default_rng(3)
    u1, u2 = rng.normal(size=len(sites)), rng.normal(size=len(sites))
    runs = [{"converged": True, "u": u1}, {"converged": True, "u": u1[perms[5]]},
            {"converged": True, "u": u2}, {"converged": False, "u": -u2},
            {"converged": True, "u": u2 * (1 + 1e-6)}, {"converged": True, "u": u1 + 0.1}]
    assert S.distinct(runs, perms) == [0, 2, 5]
