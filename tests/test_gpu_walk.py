"""Walking plane tiles (4-D problems on narrow planes, a workgroup walking
several axis-0 planes of one slab, hjr_opts.walk) against the plane tiles
one by one (walk = -1): the same arithmetic per node, so every value and
step count must be bit-identical, over grid shapes that put one or two
axis-1 slabs in a workgroup, ragged last slab groups, tiles touching every
face, walk lengths that do and do not divide axis 0, both ENO orders, both
4-D models and both precisions; plus the FP64 result against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2101_05916_amd import hjr  # noqa: E402
from paper_2101_05916_amd import workloads as W  # noqa: E402

from gpu_util import oracle_solve  # noqa: E402

pytestmark = pytest.mark.gpu

# (model, shape, order): nc <= 32 puts two axis-1 slabs in a workgroup
# (odd n1 leaves a last group of one), 33..64 one slab
SHAPES = [("x4d", (13, 13, 13, 13), 2), ("x4d", (9, 11, 17, 41), 2), ("x4d", (7, 6, 12, 61), 2),
          ("x4d", (11, 9, 21, 21), 1), ("x4dv", (9, 7, 15, 33), 2), ("x4d", (5, 5, 30, 64), 2)]


def _problem(kind, shape, order):
    return W.quad_x4dv(shape, 0.3) if kind == "x4dv" else W.quad_x4d(shape, 0.6)


def _solve(P, dtype, order, walk, steps):
    l = torch.tensor(P.l, dtype=dtype, device="cuda")
    V, st = hjr.solve(hjr.Spec.of(P), l, dtype=dtype, order=order, max_iter=steps, walk=walk,
                      tile_rows=0)
    torch.cuda.synchronize()
    return V, st


@pytest.mark.parametrize("case", SHAPES, ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[1]))}-o{c[2]}")
@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_walk_bit_identical_to_plane_tiles(case, dt):
    kind, shape, order = case
    P = _problem(kind, shape, order)
    dtype = torch.float64 if dt == "f64" else torch.float32
    steps = 20
    print(f"walk vs plane tiles: {kind} {shape} order {order} {dt}", flush=True)
    base, st0 = _solve(P, dtype, order, -1, steps)
    for walk in (1, 3, shape[0]):
        V, st = _solve(P, dtype, order, walk, steps)
        assert st["iterations"] == st0["iterations"] == steps
        assert torch.equal(V, base), (walk, float((V.double() - base.double()).abs().max()))
    if dt == "f64":
        # the plane-tile result against the oracle: 1e-16 .. 5e-14 after 20
        # steps, except 8.3e-7 on the 7 x 6 x 12 x 61 grid, where a tie
        # between two second differences of equal magnitude flips ENO2's
        # choice on rounding (the bar of the converged FP64 solves)
        ref = oracle_solve(P, order=order, max_iter=steps)
        err = float(np.max(np.abs(base.cpu().numpy() - ref["V"])))
        print(f"  fp64 vs oracle after {steps} steps: {err:.3e}")
        assert err <= 5e-5


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_walk_converged_band_solve(dt):
    """A solve to convergence over the band rule: the same stop step and
    values with walking tiles as without."""
    P = W.quad_x4d(17, 0.5, band=W.BAND_4D_UPDATE)
    dtype = torch.float64 if dt == "f64" else torch.float32
    base, st0 = _solve(P, dtype, 2, -1, 100000)
    V, st = _solve(P, dtype, 2, 4, 100000)
    assert st0["status"] == st["status"] == hjr.OK
    assert st["iterations"] == st0["iterations"]
    assert torch.equal(V, base)


def test_walk_in_batch_with_other_families():
    """Walking 4-D problems batched with 2-D and wide-plane problems: each
    result bit-identical to its single solve without walking."""
    Ps = [W.quad_x4d(15, 0.5, band=W.BAND_4D_UPDATE), W.quad_z2d(51, 0.4),
          W.quad_x4d((6, 7, 9, 70), 0.7), W.quad_x4d(12, 0.9, band=W.BAND_4D_UPDATE)]
    ls = [torch.tensor(P.l, dtype=torch.float32, device="cuda") for P in Ps]
    Vs = [torch.empty_like(l) for l in ls]
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V, tile_rows=[0]) for P, l, V in zip(Ps, ls, Vs)]
    r, stats = hjr.solve_batch(probs, dtype=torch.float32, max_iter=400, walk=2)
    torch.cuda.synchronize()
    for P, l, V, s in zip(Ps, ls, Vs, stats):
        ref, st = hjr.solve(hjr.Spec.of(P), l, dtype=torch.float32, max_iter=400, walk=-1,
                            tile_rows=0)
        torch.cuda.synchronize()
        assert s["iterations"] == st["iterations"]
        assert torch.equal(V, ref)
