"""The residual band of the 4-D stop test against solving on: the
safe set a band-stopped oracle solve returns is the one that longer solves
over every node reach.

The 4-D solves of the batched workloads stop when max |V^{k+1} - V^k| < tol
over the nodes with |V| < 0.5 (before or after the step), not over every
node: on these grids the all-node residual of ENO2 settles into a cycle
about 1e-4 high at a few nodes far from the zero level (stencil choices
flipping between steps), and some solves never meet the all-node rule.
The band rule is kept only because the sign of V, the safe set of Sec. II
eq. (2), does not depend on those nodes: here a band-stopped solve
(15^4, bound 0.5) is compared with the same problem solved from the same
cold start for four times as many steps over every node.  Measured: 449
band steps; after 1796 all-node steps 1.98e-4 of the nodes change sign
(0.1 % allowed), all within 0.011 of the zero level, while values far
from it move by up to 0.22.  (17^4 at bound 0.8: 614 steps, 7.2e-4; 31^4
mix member, 1035 band steps against 4000: 2.2e-5.)
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2101_05916_amd import workloads as W


def test_band_stopped_safe_set_matches_longer_all_node_solve():
    P = W.quad_x4d(15, 0.5, band=W.BAND_4D_UPDATE)
    g, d = O.make_grid(P.n, P.lo, P.hi), O.make_dyn(P.kind, P.params)
    a = O.solve(d, g, P.l, P.dlo, P.dhi, tol=P.tol, band=P.band)
    assert a["status"] == O.OK
    b = O.solve(d, g, P.l, P.dlo, P.dhi, tol=1e-12, max_iter=4 * a["iterations"])
    assert b["iterations"] == 4 * a["iterations"]
    A, B = a["V"], b["V"]
    flips = (A >= 0) != (B >= 0)
    assert flips.mean() <= 1e-3, flips.mean()
    # the sign changes sit at the zero level
    assert np.all(np.abs(B[flips]) <= 0.05), float(np.abs(B[flips]).max())
    # and the all-node residual of the longer solve is still not below tol
    # (the cycle the band rule steps around)
    assert b["residual"] > P.tol
