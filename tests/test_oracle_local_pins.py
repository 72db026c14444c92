"""Pins of the oracle's localized update (paper Sec. VI: localized warm
starting): a warm-started solve that updates only a band of nodes around the
zero level set of the previous value.

  band of a warm start      brute force over the straddling cells (k = 0, 1, 3)
  masked solve              all-ones mask = the full solve bit for bit; empty mask
                            stops at once; nodes outside the mask never change
  what the band buys        a small bound change on the vertical model: the band
                            update reproduces the full warm update's safe set
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2101_05916_amd import workloads as W


def og(P):
    return O.make_grid(P.n, P.lo, P.hi)


def od(P):
    return O.make_dyn(P.kind, P.params)


def band_brute(n, V, k):
    """Straddling cells by their corners' signs, then every node whose
    distance to such a cell's index range is <= k on every axis."""
    V = V.reshape(n)
    D = len(n)
    cells = []
    for c in itertools.product(*[range(x - 1) for x in n]):
        vals = [V[tuple(c[a] + o[a] for a in range(D))] for o in itertools.product((0, 1), repeat=D)]
        if min(vals) < 0 <= max(vals):
            cells.append(c)
    out = np.zeros(n, dtype=np.uint8)
    for i in itertools.product(*[range(x) for x in n]):
        for c in cells:
            if all(c[a] - k <= i[a] <= c[a] + 1 + k for a in range(D)):
                out[i] = 1
                break
    return out.ravel()


@pytest.mark.parametrize("k", [0, 1, 3])
def test_band_mask_brute_force(k):
    rng = np.random.default_rng(k)
    for n in ((9, 11), (5, 6, 4, 5)):
        G = np.meshgrid(*[np.linspace(-1, 1, x) for x in n], indexing="ij")
        V = (0.5 - sum(g * g for g in G)).ravel() + 0.01 * rng.standard_normal(int(np.prod(n)))
        P = W.Problem(W.QUAD_Z2D if len(n) == 2 else W.QUAD_X4D, (), n, (-1,) * len(n),
                      (1,) * len(n), V, (0,), (0,))
        m, cnt = O.band_mask(og(P), V, k)
        want = band_brute(n, V, k)
        assert np.array_equal(m, want) and cnt == int(want.sum())


def test_masked_all_ones_is_the_full_solve():
    for P, steps in ((W.quad_z2d(31, 0.5), 100000), (W.quad_x4d(7, 0.5), 15)):
        full = O.solve(od(P), og(P), P.l, P.dlo, P.dhi, tol=P.tol, max_iter=steps)
        loc = O.solve_masked(od(P), og(P), P.l, P.dlo, P.dhi, np.ones(P.size, np.uint8),
                             tol=P.tol, max_iter=steps)
        assert loc["iterations"] == full["iterations"]
        assert np.array_equal(loc["V"], full["V"])


def test_masked_empty_mask_and_frozen_nodes():
    P = W.quad_z2d(31, 0.5)
    rng = np.random.default_rng(4)
    V0 = P.l + 0.3 * rng.standard_normal(P.size)
    start = np.minimum(P.l, V0)
    r0 = O.solve_masked(od(P), og(P), P.l, P.dlo, P.dhi, np.zeros(P.size, np.uint8), V0=V0)
    assert r0["status"] == O.OK and r0["iterations"] == 1 and r0["residual"] == 0.0
    assert np.array_equal(r0["V"], start)
    mask = (rng.random(P.size) < 0.3).astype(np.uint8)
    r = O.solve_masked(od(P), og(P), P.l, P.dlo, P.dhi, mask, V0=V0, max_iter=50)
    assert np.array_equal(r["V"][mask == 0], start[mask == 0])
    assert np.any(r["V"][mask == 1] != start[mask == 1])


def test_band_update_reproduces_full_update():
    """Warm start from the converged value for the bound 0.5, update to
    0.55: the band of 4 cells around the old zero level set holds the new
    one, so the localized update gives the full update's safe set (to one
    node) while iterating a fraction of the grid."""
    P5, P55 = W.quad_z2d(101, 0.5), W.quad_z2d(101, 0.55)
    old = O.solve(od(P5), og(P5), P5.l, P5.dlo, P5.dhi, tol=P5.tol)["V"]
    full = O.solve(od(P55), og(P55), P55.l, P55.dlo, P55.dhi, tol=P55.tol, V0=old)
    mask, cnt = O.band_mask(og(P55), old, 4)
    loc = O.solve_masked(od(P55), og(P55), P55.l, P55.dlo, P55.dhi, mask, tol=P55.tol, V0=old)
    assert loc["status"] == O.OK
    assert cnt < 0.5 * P55.size
    assert int(np.sum((loc["V"] >= 0) != (full["V"] >= 0))) <= 1
    near = mask.astype(bool) & (np.abs(full["V"]) < 0.05)
    assert np.max(np.abs(loc["V"] - full["V"])[near]) < 1e-2
