"""Device safety queries (hjr_safety_query: value, gradient, optimal safety
control and the least-restrictive filter, paper Sec. II-A/II-B) against the
oracle's query on identical inputs.

Both sides interpolate in double from the same stored V, so value and
gradient agree to rounding (1e-12 on O(1) data); the control, an
integer-like choice on the sign of a gradient coefficient, is compared
exactly wherever that coefficient is not within 1e-9 of zero.  States
outside the grid box give NaN on both sides.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2101_05916_amd import workloads as W

from gpu_util import odyn, ogrid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_05916_amd import hjr
    hjr.lib()


def hjr_():
    from paper_2101_05916_amd import hjr
    return hjr


def states(P, n, rng):
    """Random states in the box plus its corners, points on cell faces,
    the upper box faces exactly, and a few outside or NaN."""
    lo, hi = np.array(P.lo), np.array(P.hi)
    X = lo + (hi - lo) * rng.random((n, P.ndim))
    corners = lo + (hi - lo) * ((np.arange(2 ** P.ndim)[:, None] >> np.arange(P.ndim)) & 1)
    ax = W.axes(P.n, P.lo, P.hi)
    nodes = np.array([[ax[a][rng.integers(0, P.n[a])] for a in range(P.ndim)] for _ in range(16)])
    out = np.array([lo - 0.1, hi + 0.1, np.where(np.arange(P.ndim) == 0, np.nan, lo)])
    return np.vstack([X, corners, nodes, out])


def ctrl_coef(P, grad):
    """Coefficient whose sign picks each control input."""
    p = P.params
    if P.kind == W.QUAD_Z2D:
        return (p[0] * grad[:, 1])[:, None]
    if P.kind == W.QUAD_X4D:
        return (p[3] * grad[:, 3])[:, None]
    return np.column_stack([p[0] * grad[:, int(p[9])], p[4] * grad[:, int(p[11])]])


def compare(P, V64, X, dev, order=2):
    ref = O.query(odyn(P), ogrid(P), V64, X, P.dlo, P.dhi, order=order)
    v = dev["value"].cpu().numpy()
    g = dev["grad"].cpu().numpy()
    u = dev["u_star"].cpu().numpy()
    bad = ~ref["ok"]
    assert np.array_equal(np.isnan(v), bad)
    assert np.all(np.isnan(g[bad])) and np.all(np.isnan(u[bad]))
    ok = ref["ok"]
    assert np.max(np.abs(v[ok] - ref["value"][ok])) <= 1e-12
    assert np.max(np.abs(g[ok] - ref["grad"][ok])) <= 1e-11 * max(1.0, np.abs(ref["grad"][ok]).max())
    decided = np.abs(ctrl_coef(P, ref["grad"][ok])) > 1e-9
    assert np.array_equal(u[ok][decided], ref["u"][ok][decided])
    return ref


CASES = [("z2d", (51, 51)), ("z2d", (83, 97)), ("x4d", (9, 9, 9, 9)), ("x4d", (5, 6, 7, 75)),
         ("di2x2", (6, 6, 6, 6))]


def make(kind, shape):
    if kind == "z2d":
        return W.quad_z2d(shape, 0.5)
    if kind == "x4d":
        return W.quad_x4d(shape, 0.5)
    return W.di2x2(shape[0], perm=(2, 0, 3, 1), dbar=(0.5, 0.3))


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[1]))}")
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("order", [2, 1])
def test_query_matches_oracle(case, dt, order):
    hjr = hjr_()
    P = make(*case)
    rng = np.random.default_rng(100 * order + CASES.index(case) + (7 if dt == 'f32' else 0))
    # a smooth field with structure in every axis, plus noise (no ENO ties)
    G = W.mesh(P.n, P.lo, P.hi)
    V = sum(np.sin(0.7 * (a + 1) * G[a] + a) for a in range(P.ndim)).ravel()
    V = V + 0.05 * rng.standard_normal(P.size)
    dtype = torch.float64 if dt == "f64" else torch.float32
    Vd = torch.tensor(V, dtype=dtype, device="cuda")
    V64 = Vd.cpu().numpy().astype(np.float64)  # the values the device holds
    X = states(P, 300, rng)
    out = hjr.query(hjr.Spec.of(P), Vd, torch.tensor(X, device="cuda"), order=order)
    torch.cuda.synchronize()
    compare(P, V64, X, out, order=order)


@pytest.mark.parametrize("level", [0.0, 0.2])
def test_filter_overrides_below_level(level):
    hjr = hjr_()
    P = W.quad_z2d(51, 0.5)
    r = O.solve(odyn(P), ogrid(P), P.l, P.dlo, P.dhi, tol=P.tol)
    Vd = torch.tensor(r["V"], dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(9)
    X = states(P, 500, rng)
    u_perf = rng.uniform(7.0, 16.0, (X.shape[0], 1))
    out = hjr.query(hjr.Spec.of(P), Vd, torch.tensor(X, device="cuda"),
                    u_perf=torch.tensor(u_perf, device="cuda"), level=level)
    torch.cuda.synchronize()
    v = out["value"].cpu().numpy()
    us = out["u_star"].cpu().numpy()
    uo = out["u_out"].cpu().numpy()
    keep = v >= level
    assert np.array_equal(uo[keep], u_perf[keep])
    over = ~keep & ~np.isnan(v)
    assert over.sum() > 10 and np.array_equal(uo[over], us[over])
    assert np.all(np.isnan(uo[np.isnan(v)]))


def test_query_on_device_solution_fullsize():
    """The benchmark's x-subsystem solved on the device (41^4, FP32), then
    65536 states queried in one launch; the oracle checks 400 of them."""
    hjr = hjr_()
    P = W.quad_x4d(41, 0.5)
    spec = hjr.Spec.of(P)
    V, st = hjr.solve(spec, torch.tensor(P.l, dtype=torch.float32, device="cuda"), max_iter=300)
    rng = np.random.default_rng(12)
    lo, hi = np.array(P.lo), np.array(P.hi)
    X = lo + (hi - lo) * rng.random((65536, 4))
    out = hjr.query(spec, V, torch.tensor(X, device="cuda"))
    torch.cuda.synchronize()
    V64 = V.cpu().numpy().astype(np.float64)
    pick = rng.choice(len(X), 400, replace=False)
    sub = {k: t[pick] for k, t in out.items()}
    compare(P, V64, X[pick], sub)
    # safe states (V >= 0) exist and the controller saturates (|S| = s_max)
    v = out["value"].cpu().numpy()
    assert 0.05 < np.mean(v >= 0) < 0.95
    assert np.all(np.abs(out["u_star"].cpu().numpy()) == P.params[4])
