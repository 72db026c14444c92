"""Pins of the oracle for the 10-D near-hover quadcopter as the paper writes it
(Sec. IV, eq. (3): the x and y rows take the disturbance on the velocity
rate, |S| <= 14 deg) and for decomposed queries (Sec. III-A: a decoupled
system's safe set is the product of its subsystems' sets, so its value is
their minimum and each subsystem's controller drives its own inputs).

  x-subsystem dynamics and H        the model rows; dense brute-force max-min
  LF bounds                         hand-derived maxima of |f_i|
  symmetry                          f odd, l even under x -> -x: V(x) = V(-x)
  direction of the bound            a wider disturbance bound lowers V (first order)
  decomposed query                  one subsystem = the single query; the minimum,
                                    the active subsystem, scattered gradients and
                                    controls, the per-subsystem filter, NaN outside
  decomposition safety              closed-loop rollouts of a two-subsystem system
                                    under the decomposed controller and worst-case
                                    disturbances stay in both constraint sets
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2101_05916_amd import workloads as W


def og(P):
    return O.make_grid(P.n, P.lo, P.hi)


def od(P):
    return O.make_dyn(P.kind, P.params)


SMAX = 14.0 * math.pi / 180.0


def f_x4dv(x, S, d):
    # x rows of eq. (3): disturbance on the velocity rate
    return np.array([x[1], 9.81 * math.tan(x[2]) + d, -8.0 * x[2] + x[3], -10.0 * x[2] + 10.0 * S])


def test_x4dv_dynamics_and_hamiltonian():
    P = W.quad_x4dv(5, 0.3)
    rng = np.random.default_rng(0)
    us = np.linspace(-SMAX, SMAX, 41)
    ds = np.linspace(-0.3, 0.3, 41)
    for _ in range(20):
        x = rng.uniform(-0.5, 0.5, 4)
        S, d = rng.uniform(-SMAX, SMAX), rng.uniform(-0.3, 0.3)
        assert np.allclose(O.dynamics(od(P), x, [S], [d]), f_x4dv(x, S, d), atol=1e-13)
        p = rng.standard_normal(4)
        brute = max(min(float(p @ f_x4dv(x, u, dd)) for dd in ds) for u in us)
        assert O.hamiltonian(od(P), x, p, P.dlo, P.dhi) == pytest.approx(brute, abs=1e-10)


def test_x4dv_lf_alpha():
    P = W.quad_x4dv(9, 0.3)
    a = O.lf_alpha(od(P), og(P), P.dlo, P.dhi)
    ref = [4.0, 9.81 * math.tan(math.pi / 6) + 0.3, 8 * math.pi / 6 + 4.0,
           10 * math.pi / 6 + 10 * SMAX]
    assert np.allclose(a, ref, rtol=1e-14)


def test_x4dv_symmetry():
    P = W.quad_x4dv(9, 0.3)
    r = O.solve(od(P), og(P), P.l, P.dlo, P.dhi, tol=P.tol, max_iter=40)
    assert np.max(np.abs(r["V"] - r["V"][::-1])) < 1e-10


def test_x4dv_wider_bound_lowers_value():
    """First-order LF with CFL <= 1 is monotone away from the boundary (the
    linear-extrapolation ghosts are not), so with one alpha and dt for both
    runs, a wider bound gives values <= the narrower one's at every node the
    ghosts have not reached: k steps (two stages each) move their influence
    2k nodes in."""
    P3, P6 = W.quad_x4dv(13, 0.3), W.quad_x4dv(13, 0.6)
    alpha = O.lf_alpha(od(P6), og(P6), P6.dlo, P6.dhi)
    dt = O.dt(og(P6), alpha)
    V3, V6 = P3.l.copy(), P6.l.copy()
    for k in (1, 2):
        V3, _ = O.iterate(od(P3), og(P3), P3.dlo, P3.dhi, alpha, dt, P3.l, V3, order=1)
        V6, _ = O.iterate(od(P6), og(P6), P6.dlo, P6.dhi, alpha, dt, P6.l, V6, order=1)
        inner = (slice(2 * k, 13 - 2 * k),) * 4
        a, b = V3.reshape(P3.n)[inner], V6.reshape(P6.n)[inner]
        assert np.all(b <= a + 1e-12), k
        if k == 1:
            assert np.max(a - b) > 1e-4


def sub(P, V, state_index, control_index):
    return dict(dyn=od(P), grid=og(P), V=V, state_index=list(state_index),
                control_index=control_index, dlo=P.dlo, dhi=P.dhi)


def test_decomposed_query_one_subsystem_is_the_query():
    P = W.quad_x4dv((5, 6, 7, 8), 0.3)
    rng = np.random.default_rng(1)
    V = rng.standard_normal(P.size)
    X = np.array(P.lo) + (np.array(P.hi) - np.array(P.lo)) * rng.random((50, 4))
    # the subsystem's axes are components (2, 0, 3, 1) of a 4-vector
    perm = [2, 0, 3, 1]
    Xf = np.zeros_like(X)
    Xf[:, perm] = X
    a = O.query(od(P), og(P), V, X, P.dlo, P.dhi)
    b = O.query_decomposed([sub(P, V, perm, 0)], Xf)
    assert np.array_equal(a["value"], b["value"]) and b["ok"].all()
    assert np.array_equal(a["grad"], b["grad"][:, perm])
    assert np.array_equal(a["u"], b["u"])
    assert np.all(b["active"] == 0)


def test_decomposed_query_min_active_filter():
    Px, Pz = W.quad_x4dv((5, 5, 5, 5), 0.3), W.quad_z10((9, 11), 0.3)
    rng = np.random.default_rng(2)
    Vx, Vz = rng.standard_normal(Px.size), rng.standard_normal(Pz.size)
    subs = [sub(Px, Vx, (0, 1, 2, 3), 0), sub(Px, Vx, (4, 5, 6, 7), 1), sub(Pz, Vz, (8, 9), 2)]
    lo = np.array(Px.lo * 2 + Pz.lo)
    hi = np.array(Px.hi * 2 + Pz.hi)
    X = lo + (hi - lo) * rng.random((60, 10))
    U = rng.uniform(-1, 1, (60, 3))
    q = O.query_decomposed(subs, X, level=0.1, U_perf=U)
    assert q["ok"].all()
    assert np.array_equal(q["value"], q["sub_value"].min(axis=1))
    assert np.array_equal(q["active"], q["sub_value"].argmin(axis=1))
    for k, (P, Vk, idx, c) in enumerate([(Px, Vx, [0, 1, 2, 3], 0), (Px, Vx, [4, 5, 6, 7], 1),
                                          (Pz, Vz, [8, 9], 2)]):
        s = O.query(od(P), og(P), Vk, X[:, idx], P.dlo, P.dhi)
        assert np.array_equal(q["sub_value"][:, k], s["value"])
        assert np.array_equal(q["grad"][:, idx], s["grad"])
        assert np.array_equal(q["u"][:, c], s["u"][:, 0])
        keep = s["value"] >= 0.1
        assert np.array_equal(q["u_out"][keep, c], U[keep, c])
        assert np.array_equal(q["u_out"][~keep, c], s["u"][~keep, 0])
    Xo = X[:3].copy()
    Xo[0, 9] = 9.0  # vz outside its box
    Xo[1, 2] = np.nan
    qo = O.query_decomposed(subs, Xo)
    assert list(qo["ok"]) == [False, False, True]
    assert np.isnan(qo["value"][:2]).all() and list(qo["active"][:2]) == [-1, -1]


def test_decomposed_controller_keeps_both_subsystems_safe():
    """Two vertical models (the paper's z-subsystem and the one of Sec. V)
    form one 4-D system; from states the decomposed value calls safe, the
    decomposed safety controller with each subsystem's worst-case
    disturbance keeps both altitudes inside their constraint sets."""
    A, B = W.quad_z10(51, 0.3), W.quad_z2d(51, 0.5)
    ra = O.solve(od(A), og(A), A.l, A.dlo, A.dhi, tol=A.tol)
    rb = O.solve(od(B), og(B), B.l, B.dlo, B.dhi, tol=B.tol)
    subs = [sub(A, ra["V"], (0, 1), 0), sub(B, rb["V"], (2, 3), 1)]
    rng = np.random.default_rng(3)
    lo = np.array(A.lo + B.lo)
    hi = np.array(A.hi + B.hi)
    starts = []
    while len(starts) < 12:
        x = lo + (hi - lo) * rng.random(4)
        if O.query_decomposed(subs, x[None])["value"][0] > 0.15:
            starts.append(x)

    def f(x, u, d):
        return np.array([x[1], A.params[0] * u[0] - 9.81 + d[0],
                         x[3], B.params[0] * u[1] - 9.81 + d[1]])

    dt = 4e-3
    for x in starts:
        v0 = O.query_decomposed(subs, x[None])["value"][0]
        lmin = np.inf
        for _ in range(500):
            q = O.query_decomposed(subs, x[None])
            u = q["u"][0]
            g = q["grad"][0]
            d = np.array([-0.3 if g[1] >= 0 else 0.3, -0.5 if g[3] >= 0 else 0.5])
            k1 = f(x, u, d)
            k2 = f(x + 0.5 * dt * k1, u, d)
            k3 = f(x + 0.5 * dt * k2, u, d)
            k4 = f(x + dt * k3, u, d)
            x = x + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            la = min(x[0] - 0.35, 2.8 - x[0], 3.5 - abs(x[1]))
            lb = min(x[2] - 0.5, 2.5 - x[2])
            lmin = min(lmin, la, lb)
        assert lmin > 0 and lmin >= v0 - 0.15
