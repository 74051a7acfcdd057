"""Planted mistakes: each test loads a copy of the oracle's walker with one
plausible mistake written into its source (on the CPU, in memory; the
oracle itself is untouched) and checks that the closed-form pins fail for
it.  This is the evidence that the pins constrain where and how much each
walk tallies, not only the row sums.

Mistakes planted (each a one-line change of oracle/walker.py):
  chain tally point X_k instead of X_k + r_k Y     -> T7 (A), T8
  k = 0 tally at x instead of x + r0 Y              -> T7 (A)
  ball term of B at x + r0 Zs (S dropped)           -> T7 (B)
  d = 2 weight omega dropped                        -> T7 (A)
  sign of the chain term of B flipped               -> T7 (B)
  terminal point taken at the start                 -> T9 (H)
  K weight along Zs instead of U1                   -> T9 (K)
"""
import os
import types

import numpy as np
import pytest

import workloads as W

from test_oracle_green_pins import t7_zscores, t8_zscore, t9_zscore, _disk_ball_phi

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "walker.py")


def mutant(old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "the planted line is no longer in oracle/walker.py: " + old
    mod = types.ModuleType("oracle._mutant_walker")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), "<oracle/walker.py, mutated>", "exec"), mod.__dict__)
    return mod


MUTANTS = {
    "tally_at_X": ("pts.append(X[a] + r[:, None] * Y[a])", "pts.append(X[a].copy())"),
    "k0_at_x": ("[x + r0 * Y]", "[x + 0.0 * Y]"),
    "ball_term_without_S": ("ev.ball_pts = x + r0 * S[:, None] * Zs", "ev.ball_pts = x + r0 * Zs"),
    "omega_dropped": ("om = np.ones_like(R) if exact else omega(R, d)", "om = np.ones_like(R)"),
    "B_chain_sign": ("tB.append(t[:, None] * w[a])", "tB.append(-t[:, None] * w[a])"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_t7_catches_the_planted_mistake(name):
    mod = mutant(*MUTANTS[name])
    # dropping omega moves about a fifth of the chain mass spread over all
    # cells, so it needs the pin's full walk count to stand out per entry
    walks = 200000 if name == "omega_dropped" else 40000
    assert t7_zscores(mod, 2, rows=(2,), walks=walks) > 3.0


def test_t8_catches_the_tally_point_at_X():
    # a non-harmonic source tells X_k + r_k Y from X_k
    mod = mutant(*MUTANTS["tally_at_X"])
    assert t8_zscore(mod, W.unit_disk(), _disk_ball_phi(2), [[0.35, -0.2]], N=20000) > 3.0


@pytest.mark.parametrize("old,new", [
    ("    ev.term_pts = X\n", "    ev.term_pts = x + 0.0 * X\n"),   # exit point = start point
    ("    w = (d / r0) * U1\n", "    w = (d / r0) * Zs\n"),          # K weight from the wrong direction
], ids=["terminal_at_start", "K_weight_direction"])
def test_t9_catches_the_planted_mistake(old, new):
    assert t9_zscore(mutant(old, new), N=20000) > 3.0


def test_the_unmutated_copy_passes():
    # the loader itself changes nothing
    mod = mutant("DEFAULT_MAX_STEPS = 10000", "DEFAULT_MAX_STEPS = 10000")
    assert t7_zscores(mod, 2, rows=(2,), walks=40000) <= 1.0
