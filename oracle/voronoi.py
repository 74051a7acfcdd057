"""Nearest-centre maps (oracle).

The toolbox never stores Voronoi cells: membership 1_{V_j}(q) is
"q's nearest centre is y_j" (Sec. "Matrix estimators", Voronoi example,
and Rem. "implementation_tips" (iii)).  Here it is the plain definition,
argmin_j |q - y_j|, by brute force in FP64; ties go to the lowest index
(numpy argmin semantics).  The query set is processed in slices only to
bound memory.

Pinned by tests/test_oracle_voronoi.py (regular lattices whose nearest
centre is known in closed form, and exact ties).
"""
import numpy as np


def nearest(centres, q):
    centres = np.asarray(centres, dtype=np.float64)
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    out = np.empty(len(q), dtype=np.int64)
    chunk = max(1, 4_000_000 // (centres.shape[0] * centres.shape[1]))
    for s in range(0, len(q), chunk):
        qq = q[s:s + chunk]
        # |q - y|^2 computed directly (no expansion) so that exact ties stay ties
        d2 = ((qq[:, None, :] - centres[None, :, :]) ** 2).sum(axis=2)
        out[s:s + chunk] = np.argmin(d2, axis=1)
    return out
