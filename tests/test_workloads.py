"""The seeded input recipes (no method arithmetic lives there)."""
import numpy as np

import workloads as W


def test_served_problem_is_consistent():
    cfg = W.config("lshape256")
    x, z = cfg["sites"], cfg["bnodes"]
    P = W.anisotropic_problem(7, x, z)
    ev = np.linalg.eigvalsh(P["A"])
    assert ev.min() > 0.99 and ev.max() < 100.01          # SPD, anisotropy <= 1:100
    assert np.all(np.linalg.norm(P["b"], axis=1) <= 0.8 + 1e-12)
    # the derived source does not depend on the difference step
    P2 = W.anisotropic_problem(7, x, z, h=2e-5)
    assert np.allclose(P["f"], P2["f"], rtol=1e-6, atol=1e-6 * np.abs(P["f"]).max())
    # same seed, same problem; another seed, another one
    assert np.array_equal(W.anisotropic_problem(7, x, z)["f"], P["f"])
    assert not np.allclose(W.anisotropic_problem(8, x, z)["f"], P["f"])


def test_served_problem_source_for_constant_coefficients():
    # with A = I and b = 0 the flux divergence is the Laplacian: pin the
    # finite-difference divergence against the closed-form Laplacian
    u, gu, lap = W.smooth_field(3, 2, terms=5, max_freq=2.0)
    x = np.random.default_rng(0).uniform(-0.5, 0.5, (50, 2))
    h = 1e-5
    div = sum((gu(x + h * e)[:, a] - gu(x - h * e)[:, a]) / (2 * h) for a, e in enumerate(np.eye(2)))
    assert np.allclose(div, lap(x), rtol=1e-6, atol=1e-7)


def test_torsion_exact_solution_matches_the_oracle():
    from oracle.euler_lagrange import plaplace_torsion_disk
    x = np.random.default_rng(1).uniform(-0.7, 0.7, size=(50, 2))
    for P in (1.5, 2.0, 5.0, 50.0):
        assert np.allclose(W.plaplace_torsion_disk_exact(x, P), plaplace_torsion_disk(x, P), rtol=1e-14, atol=0)
