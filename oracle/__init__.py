"""CPU oracle for the extended Walk-on-Spheres operator toolbox.

This package is TEST INFRASTRUCTURE.  It is a plain, slow, FP64 NumPy
implementation of what the GPU path computes, written from the paper
(Cimpean, Grecu, Zarnescu, "Extended Walk-on-Spheres Algorithm for Linear and
Nonlinear Elliptic Problems of Divergence-type"):

* ``philox``    -- the counter-based generator both sides draw from
                   (Philox4x32-10, from its published definition);
* ``geometry``  -- distance to the boundary r(x), eq. (r), and inside tests;
* ``samplers``  -- the refined samplers of Prop. "removing singularities"
                   and Rem. "MC_no_singular";
* ``voronoi``   -- brute-force nearest-centre maps (Sec. "Matrix estimators",
                   Voronoi example);
* ``walker``    -- the per-walk events of Alg. "WoS-LOT" and the binned
                   toolbox A, B, H, K (eqs. Estimator_A/B/H/K) plus the
                   pointwise estimators (eqs. u MC, gradu U MC, H MC, dh MC);
* ``volume``    -- the cell weights lambda_i = |W_i| / |D|;
* ``linalg``    -- assembly of Lambda, Sigma and the right-hand side
                   (eq. linear_q), the truncated-SVD solve, reconstruction,
                   and the Newton / Picard outer loops;
* ``euler_lagrange`` -- the discrete functional J of eq. gradJ for the
                   p-Laplace energy, its gradient, and Adam (Sec.
                   "Euler-Lagrange boundary value problems" and the
                   appendix on the optimisation of J).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (``paper_2608_07017_amd``)
never imports it, and it never imports the product path: the two share no
code.  The only shared module is ``workloads`` (seeded input generators,
none of the method's arithmetic).

Parity status of each function is stated in its module header.  Every
function here is pinned by a ``-m "not gpu"`` test against a closed form,
an exact invariant, brute force, or a library routine; none is marked
"parity unpinned".
"""
