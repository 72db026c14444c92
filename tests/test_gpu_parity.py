"""Device solves against the FP64 oracle, element by element, on identical
seeded inputs.

Bars: FP64 device path max|dV| <= FP64_TOL and identical step counts; FP32
device path max|dV| <= 1e-4, zero-level-set disagreement <= 0.1 % of nodes,
step counts identical (+-1 only when the oracle's stopping residual lies
within 1e-3 relative of tol); dt within 4 ulp.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2101_05916_amd import workloads as W

from gpu_util import (device_solve, iterations_match, odyn, ogrid, oracle_solve,
                      zero_level_disagreement)

pytestmark = pytest.mark.gpu

# FP64 device vs FP64 oracle: both evaluate the same formulas in a
# different order (raw differences scaled once by 1/h, fused multiply-adds,
# closed-form vs vertex-enumerated Hamiltonian), and ENO2's choice between two
# second differences is a discontinuous function of the data wherever they
# tie in magnitude (e.g. on the ghost-extended boundary lines), so rounding
# can switch the stencil at a node.  The oracle alone moves by up to 3.9e-6
# when its constraint array is perturbed by +-1 ulp (pinned in
# test_oracle_pins.py::test_rounding_sensitivity_of_the_scheme); an
# evaluation-order change perturbs every operation, so the bar allows an
# order of magnitude more and stays below the FP32 bar.
FP64_TOL = 5e-5
# FP64 runs of a fixed, small number of steps (<= 40 ENO2 steps, or first-order
# steps, which make no stencil choice): too few steps for a stencil flip to be
# likely, so the two evaluation orders agree to rounding, ~1e-14 (13^4 band
# solve: 1.6e-14; 21^4 after 40 steps: ~1e-14).  A constant wrong at the 1e-6
# level fails this bar.
FP64_STEP_TOL = 1e-10

torch = pytest.importorskip("torch")


def _ulps(a, b):
    return abs(a - b) / np.spacing(max(abs(a), abs(b)))


@pytest.fixture(scope="module", autouse=True)
def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_05916_amd import hjr
    hjr.lib()


# ---------------------------------------------------------------- 2-D, full solves

@pytest.mark.parametrize("n,dbar", [(51, 0.5), (101, 0.5), (101, 0.0), (101, 0.8)])
def test_z2d_fp64_full_solve(n, dbar):
    P = W.quad_z2d(n, dbar)
    ref = oracle_solve(P, history=True)
    V, st = device_solve(P, torch.float64)
    print(f"z2d {n} d={dbar} fp64: it {st['iterations']} vs {ref['iterations']}")
    assert st["status"] == 0 and ref["status"] == 0
    assert st["iterations"] == ref["iterations"]
    assert _ulps(st["dt"], ref["dt"]) <= 4
    assert np.max(np.abs(V - ref["V"])) <= FP64_TOL
    assert abs(st["residual"] - ref["residual"]) <= FP64_TOL


@pytest.mark.parametrize("n,dbar", [(51, 0.5), (101, 0.5), (201, 0.5)])
def test_z2d_fp32_full_solve(n, dbar):
    P = W.quad_z2d(n, dbar)
    ref = oracle_solve(P, history=True)
    V, st = device_solve(P, torch.float32)
    err = float(np.max(np.abs(V - ref["V"])))
    dis = zero_level_disagreement(V, ref["V"])
    print(f"z2d {n} fp32: it {st['iterations']} vs {ref['iterations']}, "
          f"max|dV| {err:.3e}, zero-level disagreement {dis:.2e}")
    assert st["status"] == 0
    assert iterations_match(st["iterations"], ref)
    assert err <= 1e-4
    assert dis <= 1e-3


# ---------------------------------------------------------------- narrow-band stop rule

@pytest.mark.parametrize("case", ["x4d13_f64", "x4d13_f32", "z2d101_f64"])
def test_band_full_solve(case):
    """Stop test over the band |V| < 0.5: the device stops at the oracle's
    step (13^4 has ragged LDS tiles; the band cuts 1175 steps to 410)."""
    kind, dt = case.split("_")
    P = W.quad_x4d(13, 0.5, band=0.5) if kind == "x4d13" else W.quad_z2d(101, 0.5)
    if kind == "z2d101":
        P.band = 0.5
    ref = oracle_solve(P, history=True)
    V, st = device_solve(P, torch.float64 if dt == "f64" else torch.float32)
    err = float(np.max(np.abs(V - ref["V"])))
    dis = zero_level_disagreement(V, ref["V"])
    print(f"{case} band 0.5: it {st['iterations']} vs {ref['iterations']}, max|dV| {err:.3e}, "
          f"zero-level disagreement {dis:.2e}")
    assert st["status"] == 0 and ref["status"] == 0
    if dt == "f64":
        assert st["iterations"] == ref["iterations"]
        assert err <= FP64_TOL
    else:
        assert iterations_match(st["iterations"], ref)
        assert err <= 1e-4
        assert dis <= 1e-3


# ---------------------------------------------------------------- 4-D, fixed step counts

def _x4d_fixed(n, dtype, steps, dbar=0.5):
    P = W.quad_x4d(n, dbar)
    ref = oracle_solve(P, max_iter=steps)
    V, st = device_solve(P, dtype, max_iter=steps)
    assert st["status"] == 3 and ref["status"] == 3  # NOT_CONVERGED after `steps`
    assert st["iterations"] == steps == ref["iterations"]
    return V, st, ref


def test_x4d_fp64_21_steps40():
    V, st, ref = _x4d_fixed(21, torch.float64, 40)
    assert _ulps(st["dt"], ref["dt"]) <= 4
    for a in range(4):
        assert _ulps(st["alpha"][a], ref["alpha"][a]) <= 4
    err = float(np.max(np.abs(V - ref["V"])))
    print(f"x4d 21^4 fp64 40 steps: max|dV| {err:.3e}")
    assert err <= FP64_STEP_TOL


def test_x4d_fp32_21_steps40():
    V, st, ref = _x4d_fixed(21, torch.float32, 40)
    err = float(np.max(np.abs(V - ref["V"])))
    print(f"x4d 21^4 fp32 40 steps: max|dV| {err:.3e}")
    assert err <= 1e-4


def test_x4d_fp64_ragged_shape():
    # non-cubic grid: every axis has its own length and stride, and the
    # flat size is not a multiple of the tile
    P = W.quad_x4d((9, 13, 11, 15), 0.5)
    ref = oracle_solve(P, max_iter=25)
    V, st = device_solve(P, torch.float64, max_iter=25)
    assert st["iterations"] == ref["iterations"] == 25
    err = float(np.max(np.abs(V - ref["V"])))
    print(f"x4d ragged fp64 25 steps: max|dV| {err:.3e}")
    assert err <= FP64_STEP_TOL


@pytest.mark.parametrize("perm", [(0, 1, 2, 3), (3, 1, 0, 2), (2, 0, 1, 3)])
def test_di2x2_fp64_axis_permutations(perm):
    # the same pair of 2-D models with its coordinates on different axes:
    # exercises every stride of the 4-D stencil
    P = W.di2x2((11, 12, 13, 14), perm=perm)
    ref = oracle_solve(P, max_iter=30)
    V, st = device_solve(P, torch.float64, max_iter=30)
    err = float(np.max(np.abs(V - ref["V"])))
    print(f"di2x2 {perm} fp64 30 steps: max|dV| {err:.3e}")
    # the two copies of the vertical model give second differences of equal
    # magnitude in many places, where ENO2's choice flips on rounding: with
    # the coordinates on axes (0, 1, 2, 3) the device and the oracle differ
    # by 1.1e-7 after 30 steps (6.7e-15 in the other two layouts)
    assert err <= FP64_TOL


def test_minimal_grid_n3():
    P = W.quad_z2d((3, 3), 0.5)
    ref = oracle_solve(P, max_iter=50)
    V, st = device_solve(P, torch.float64, max_iter=50)
    assert st["iterations"] == ref["iterations"]
    assert np.max(np.abs(V - ref["V"])) <= FP64_TOL


def test_first_order_matches_oracle():
    P = W.quad_z2d(41, 0.5)
    ref = oracle_solve(P, order=1, max_iter=300)
    V, st = device_solve(P, torch.float64, order=1, max_iter=300)
    assert st["iterations"] == ref["iterations"]
    err = float(np.max(np.abs(V - ref["V"])))
    print(f"z2d 41^2 first order fp64 {st['iterations']} steps: max|dV| {err:.3e}")
    assert err <= FP64_STEP_TOL


# ---------------------------------------------------------------- every tile family

# (shape, order): the plane-tile families the configurations above leave out
# -- 4-D planes wider than 68 nodes (row stride 208), and first-order 4-D and
# wide 2-D planes -- each with tiles whose node count is not a multiple of 4
# (the FP32 16-byte stage-2 tile's partial quad)
FAMILY_CASES = [("x4d", (5, 6, 7, 75), 2), ("x4d", (5, 6, 7, 75), 1), ("x4d", (9, 11, 13, 15), 1),
                ("z2d", (83, 97), 1), ("x4d", (4, 5, 11, 69), 2)]


@pytest.mark.parametrize("case", FAMILY_CASES, ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[1]))}-o{c[2]}")
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_tile_families_match_oracle(case, dt):
    kind, shape, order = case
    P = W.quad_x4d(shape, 0.6) if kind == "x4d" else W.quad_z2d(shape, 0.6)
    steps = 30
    ref = oracle_solve(P, order=order, max_iter=steps)
    V, st = device_solve(P, torch.float64 if dt == "f64" else torch.float32, order=order,
                         max_iter=steps)
    err = float(np.max(np.abs(V - ref["V"])))
    print(f"{kind} {shape} order {order} {dt}: {steps} steps, max|dV| {err:.3e}")
    assert st["iterations"] == ref["iterations"] == steps
    assert err <= (FP64_STEP_TOL if dt == "f64" else 1e-4)


# ---------------------------------------------------------------- warm start

def test_warm_start_fp64_matches_oracle():
    P5 = W.quad_z2d(101, 0.5)
    r5 = oracle_solve(P5)
    P8 = W.quad_z2d(101, 0.8)
    ref = oracle_solve(P8, V0=r5["V"])
    V, st = device_solve(P8, torch.float64, V0=r5["V"])
    assert st["iterations"] == ref["iterations"]
    assert np.max(np.abs(V - ref["V"])) <= FP64_TOL


# ---------------------------------------------------------------- chunking modes

@pytest.mark.parametrize("flags,chunk", [(0, 0), (1, 0), (2, 0), (3, 7), (4, 0), (0, 1), (8, 0)])
def test_launch_modes_bit_identical(flags, chunk):
    from paper_2101_05916_amd import hjr
    P = W.quad_z2d(61, 0.5)
    base, st0 = device_solve(P, torch.float32)
    V, st = device_solve(P, torch.float32, flags=flags, chunk=chunk)
    assert st["iterations"] == st0["iterations"]
    if flags & hjr.FLAG_FLAT_TILES:
        # the flat tiles evaluate the same arithmetic through other ghost
        # code: equal up to FP32 rounding, not bit for bit
        assert np.max(np.abs(V - base)) <= 1e-4
    else:
        assert np.array_equal(V, base)
    if flags & hjr.FLAG_PROFILE:
        assert st["kernel_launches"][0] > 0 and st["kernel_ms"][1] > 0


# ---------------------------------------------------------------- full-size sampled

@pytest.mark.parametrize("n", [41, 61, 81])
def test_x4d_fullsize_sampled_step(n):
    """At the benchmark sizes (and 81^4, whose 81-node planes take the wide
    LDS tiles): run k device steps, then one more, and check the last step
    at sampled nodes (all corners and edges included) against the oracle's
    single-node step from the device's own V_k."""
    import torch as T
    from paper_2101_05916_amd import hjr
    P = W.quad_x4d(n, 0.5)
    spec = hjr.Spec.of(P)
    l = T.tensor(P.l, dtype=T.float32, device="cuda")
    k = 15
    Vk, stk = hjr.solve(spec, l, dtype=T.float32, max_iter=k)
    Vk1, stk1 = hjr.solve(spec, l, V0=Vk.clone(), dtype=T.float32, max_iter=1)
    T.cuda.synchronize()
    a = Vk.cpu().numpy().astype(np.float64)
    b = Vk1.cpu().numpy().astype(np.float64)
    g, d = ogrid(P), odyn(P)
    alpha = O.lf_alpha(d, g, P.dlo, P.dhi)
    dt = O.dt(g, alpha)
    rng = np.random.default_rng(7)
    N = P.size
    corners = [np.ravel_multi_index(tuple((n - 1) * ((c >> i) & 1) for i in range(4)), P.n)
               for c in range(16)]
    edge = [np.ravel_multi_index((0, 1, n - 2, n // 2), P.n), np.ravel_multi_index((1, 0, 0, 1), P.n)]
    idx = np.concatenate([corners, edge, rng.integers(0, N, 400)])
    worst = 0.0
    for i in idx:
        v = O.iterate_at(d, g, P.dlo, P.dhi, alpha, dt, P.l, a, int(i))
        worst = max(worst, abs(v - b[i]))
    print(f"x4d {n}^4 sampled single-step max|dV| {worst:.3e}")
    assert worst <= 2e-6


# ---------------------------------------------------------------- interpolation & mask

@pytest.mark.parametrize("case", [("2d", 51, 101), ("4d", 21, 41), ("4d", 41, 61),
                                  ("4d", 61, 21), ("2d", 101, 101)])
def test_interp_bit_exact(case):
    from paper_2101_05916_amd import hjr
    kind, ns, nd = case
    P = W.quad_x4d(ns) if kind == "4d" else W.quad_z2d(ns)
    Q = W.quad_x4d(nd) if kind == "4d" else W.quad_z2d(nd)
    rng = np.random.default_rng(3)
    Vs = rng.standard_normal(P.size).astype(np.float32)
    out = hjr.interp(P.n, torch.tensor(Vs, device="cuda"), Q.n, P.lo, P.hi)
    ref = O.interp(ogrid(P), Vs.astype(np.float64), ogrid(Q)).astype(np.float32)
    assert np.array_equal(out.cpu().numpy(), ref)
    # with the projection onto the finer constraint
    lq = torch.tensor(Q.l, dtype=torch.float32, device="cuda")
    out2 = hjr.interp(P.n, torch.tensor(Vs, device="cuda"), Q.n, P.lo, P.hi, l_dst=lq)
    lf = Q.l.astype(np.float32)
    assert np.array_equal(out2.cpu().numpy(), np.where(lf < ref, lf, ref))


@pytest.mark.parametrize("n,ndim", [(101, 2), (21, 4), (41, 4)])
def test_mask_bit_exact(n, ndim):
    from paper_2101_05916_amd import hjr
    P = W.quad_x4d(n) if ndim == 4 else W.quad_z2d(n)
    rng = np.random.default_rng(5)
    V = (P.l + 0.3 * rng.standard_normal(P.size)).astype(np.float32)
    V[::7] = 0.0  # exact zeros count as safe
    m, cnt = hjr.refine_mask(P.n, P.lo, P.hi, torch.tensor(V, device="cuda"))
    ref, rc = O.refine_mask(ogrid(P), V.astype(np.float64))
    assert cnt == rc
    assert np.array_equal(m.cpu().numpy(), ref)


@pytest.mark.parametrize("shape,kind", [((21, 21, 21, 21), "x4d"), ((9, 13, 11, 15), "x4d"),
                                        ((101, 101), "z2d"), ((40, 230), "z2d")])
def test_flat_tiles_match_oracle(shape, kind):
    """The shape-agnostic fallback tiles, forced on shapes that normally take
    the LDS plane tiles, and on a 2-D grid too wide for them (230 nodes)."""
    from paper_2101_05916_amd import hjr
    P = W.quad_x4d(shape, 0.5) if kind == "x4d" else W.quad_z2d(shape, 0.5)
    ref = oracle_solve(P, max_iter=30)
    for flags in (0, hjr.FLAG_FLAT_TILES):
        V, st = device_solve(P, torch.float64, max_iter=30, flags=flags)
        assert st["iterations"] == 30
        err = float(np.max(np.abs(V - ref["V"])))
        print(f"{kind} {shape} flags {flags} fp64 30 steps: max|dV| {err:.3e}")
        assert err <= FP64_STEP_TOL
