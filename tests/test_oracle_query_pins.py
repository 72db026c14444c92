"""Pins of the oracle's safety query (paper Sec. II-A: the gradient of the
converged value function yields the optimal safety controller; Sec. II-B:
the safety controller overrides the learned policy near the boundary of the
safe set).

  value (multilinear interpolation)   exact on multilinear V; node values
  gradient (ENO node gradients,        exact on linear V (ghosts included) and on
  interpolated)                        quadratics away from the boundary
  u* (Hamiltonian's optimiser)         braking-curve closed form of the vertical
                                       model, sign rules of the x-subsystem, ties
  safety of u* (Sec. II-A)             closed-loop rollouts with the worst-case
                                       disturbance stay in the constraint set
  outside the grid box                 NaN outputs, EINVAL
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2101_05916_amd import workloads as W


def og(P):
    return O.make_grid(P.n, P.lo, P.hi)


def od(P):
    return O.make_dyn(P.kind, P.params)


def random_states(P, n, rng, margin=0.0):
    lo, hi = np.array(P.lo), np.array(P.hi)
    span = hi - lo
    return lo + margin * span + (1 - 2 * margin) * span * rng.random((n, P.ndim))


CASES = [W.quad_z2d((11, 13), 0.5), W.quad_x4d((5, 6, 7, 8), 0.5),
         W.di2x2(6, perm=(2, 0, 3, 1), dbar=(0.5, 0.3))]


@pytest.mark.parametrize("P", CASES, ids=lambda P: P.name)
def test_linear_value_exact(P):
    rng = np.random.default_rng(1)
    a = rng.standard_normal(P.ndim)
    G = W.mesh(P.n, P.lo, P.hi)
    V = (0.3 + sum(a[i] * G[i] for i in range(P.ndim))).ravel()
    X = random_states(P, 200, rng)
    X[:8] = np.array(P.lo) + (np.array(P.hi) - np.array(P.lo)) * (
        (np.arange(8)[:, None] >> np.arange(P.ndim)) & 1)  # box corners
    q = O.query(od(P), og(P), V, X, P.dlo, P.dhi)
    assert q["ok"].all()
    assert np.allclose(q["value"], 0.3 + X @ a, atol=1e-12)
    assert np.allclose(q["grad"], np.broadcast_to(a, q["grad"].shape), atol=1e-11)


def test_value_at_nodes_and_cell_centres():
    P = W.quad_x4d((5, 6, 7, 8), 0.5)
    rng = np.random.default_rng(2)
    V = rng.standard_normal(P.size)
    ax = W.axes(P.n, P.lo, P.hi)
    Vg = V.reshape(P.n)
    idx = [tuple(rng.integers(0, n - 1) for n in P.n) for _ in range(20)]
    X = np.array([[ax[i][j[i]] for i in range(4)] for j in idx])
    q = O.query(od(P), og(P), V, X, P.dlo, P.dhi)
    assert np.allclose(q["value"], [Vg[j] for j in idx], atol=1e-14)
    # cell centre: the mean of the 16 corner values
    Xc = np.array([[0.5 * (ax[i][j[i]] + ax[i][j[i] + 1]) for i in range(4)] for j in idx])
    qc = O.query(od(P), og(P), V, Xc, P.dlo, P.dhi)
    want = [np.mean(Vg[j[0]:j[0] + 2, j[1]:j[1] + 2, j[2]:j[2] + 2, j[3]:j[3] + 2]) for j in idx]
    assert np.allclose(qc["value"], want, atol=1e-14)


def test_gradient_of_quadratic_interior():
    """ENO2 is exact on quadratics at interior nodes, and the multilinear
    interpolation of the exact (linear) gradient is exact."""
    P = W.quad_z2d((21, 25), 0.5)
    Z, VZ = W.mesh(P.n, P.lo, P.hi)
    V = (0.7 * Z ** 2 - 0.2 * VZ ** 2 + 0.1 * VZ).ravel()
    rng = np.random.default_rng(3)
    hz, hv = 3 / 20, 8 / 24
    X = np.column_stack([rng.uniform(2 * hz, 3 - 3 * hz, 100), rng.uniform(-4 + 2 * hv, 4 - 3 * hv, 100)])
    q = O.query(od(P), og(P), V, X, P.dlo, P.dhi)
    assert np.allclose(q["grad"][:, 0], 1.4 * X[:, 0], atol=1e-12)
    assert np.allclose(q["grad"][:, 1], -0.4 * X[:, 1] + 0.1, atol=1e-12)


def closed_form_z2d(Z, VZ, dbar):
    a_up, a_dn = 0.91 * 16 - 9.81 - dbar, 9.81 - 0.91 * 7 - dbar
    down = np.minimum(Z - 0.5 - VZ ** 2 / (2 * a_up), 2.5 - Z)
    up = np.minimum(Z - 0.5, 2.5 - Z - VZ ** 2 / (2 * a_dn))
    return np.where(VZ <= 0, down, up)


def test_controller_on_braking_closed_form():
    """On the closed-form value of the vertical model: falling toward the
    floor (the lower braking branch decides V) the controller applies full
    thrust; rising toward the ceiling it applies the least thrust."""
    P = W.quad_z2d(101, 0.5)
    Z, VZ = W.mesh(P.n, P.lo, P.hi)
    V = closed_form_z2d(Z, VZ, 0.5).ravel()
    rng = np.random.default_rng(4)
    fall = np.column_stack([rng.uniform(0.7, 1.2, 50), rng.uniform(-3.0, -0.5, 50)])
    rise = np.column_stack([rng.uniform(1.8, 2.3, 50), rng.uniform(0.5, 3.0, 50)])
    # keep states whose value is set by the braking term (away from the kink)
    qf = O.query(od(P), og(P), V, fall, P.dlo, P.dhi)
    qr = O.query(od(P), og(P), V, rise, P.dlo, P.dhi)
    assert np.all(qf["u"][:, 0] == 16.0)
    assert np.all(qr["u"][:, 0] == 7.0)
    assert np.all(qf["grad"][:, 1] > 0) and np.all(qr["grad"][:, 1] < 0)


def test_x4d_control_sign_and_ties():
    P = W.quad_x4d((5, 5, 5, 5), 0.5)
    G = W.mesh(P.n, P.lo, P.hi)
    rng = np.random.default_rng(5)
    X = random_states(P, 30, rng)
    smax = P.params[4]
    up = O.query(od(P), og(P), (0.2 * G[3]).ravel(), X, P.dlo, P.dhi)
    dn = O.query(od(P), og(P), (-0.2 * G[3] + G[0]).ravel(), X, P.dlo, P.dhi)
    tie = O.query(od(P), og(P), (G[0] - G[1]).ravel(), X, P.dlo, P.dhi)  # no omega dependence
    assert np.all(up["u"][:, 0] == smax)
    assert np.all(dn["u"][:, 0] == -smax)
    assert np.all(tie["u"][:, 0] == smax)  # a tie takes the upper bound


def test_di2x2_controls_per_copy():
    P = W.di2x2(6, perm=(0, 1, 2, 3), dbar=(0.5, 0.3))
    G = W.mesh(P.n, P.lo, P.hi)
    rng = np.random.default_rng(6)
    X = random_states(P, 20, rng)
    q = O.query(od(P), og(P), (G[1] - G[3]).ravel(), X, P.dlo, P.dhi)  # dV/dv_a > 0, dV/dv_b < 0
    assert np.all(q["u"][:, 0] == 16.0) and np.all(q["u"][:, 1] == 7.0)


def test_outside_box_is_nan():
    P = W.quad_z2d(11, 0.5)
    V = np.zeros(P.size)
    q = O.query(od(P), og(P), V, [[3.01, 0.0], [1.0, -4.5], [np.nan, 0.0], [3.0, 4.0]], P.dlo, P.dhi)
    assert list(q["ok"]) == [False, False, False, True]
    assert np.isnan(q["value"][:3]).all() and np.isnan(q["u"][:3]).all()


def test_query_controller_keeps_states_safe():
    """Sec. II-A: from a state the converged value calls safe, the optimal
    safety controller keeps the system in the constraint set against the
    worst-case disturbance (closed loop with the query's u*, RK4, the
    disturbance at the bound that opposes the controller)."""
    P = W.quad_z2d(51, 0.5)
    r = O.solve(od(P), og(P), P.l, P.dlo, P.dhi, tol=P.tol)
    V = r["V"]
    Vg = V.reshape(P.n)
    zs, vs = W.axes(P.n, P.lo, P.hi)
    rng = np.random.default_rng(8)
    idx = np.argwhere(Vg > 0.15)
    pick = idx[rng.choice(len(idx), 20, replace=False)]

    def f(x, u, d):
        return np.array([x[1], 0.91 * u - 9.81 + d])

    dt = 4e-3
    for i, j in pick:
        x = np.array([zs[i], vs[j]])
        lmin = np.inf
        for _ in range(600):
            q = O.query(od(P), og(P), V, x[None], P.dlo, P.dhi)
            u = q["u"][0, 0]
            d = -0.5 if q["grad"][0, 1] >= 0 else 0.5
            k1 = f(x, u, d)
            k2 = f(x + 0.5 * dt * k1, u, d)
            k3 = f(x + 0.5 * dt * k2, u, d)
            k4 = f(x + dt * k3, u, d)
            x = x + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            lmin = min(lmin, min(x[0] - 0.5, 2.5 - x[0]))
        assert lmin >= Vg[i, j] - 0.15
        assert lmin > 0
