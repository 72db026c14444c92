"""Rollout pins of the oracle's converged value (paper Sec. II-A, eq. (1): V at
a state is the best margin min_t l(xi(t)) a controller can keep from it
against the worst disturbance).  Forward simulation of the models under
controls and disturbances read off the oracle's V, independent of the
scheme that computed V:

  * lower bound (4-D x-subsystem, 2-D vertical model): under the safety
    controller u* (the control-box vertex maximising grad V . f) the margin
    kept against the adversarial disturbance d* = argmin_d grad V . f, the
    two constant extremes and a disturbance switching at random every 0.1 s
    is at least V(x0) - eps;
  * unsafe side (4-D): from states with V(x0) < 0 the adversarial play
    drives the state out of the constraint set, min_t l <= V(x0) + eps;
  * upper bound (2-D): no bang-bang control with at most one switch keeps
    a larger margin against d* than V(x0) + eps, and eps shrinks when the
    grid is refined.

These check the sign structure of V against the model's own dynamics,
not parity: on grids this coarse the dissipation of the scheme makes V
conservative (the controlled trajectories keep up to ~0.1 more than V), so
the lower bound has slack, and the upper bound (2-D) and the unsafe side
(4-D) are what tie V to the dynamics from above.

Integration: classical RK4, 1 ms steps, over 3 s (4-D) or 2 s (2-D); the
gradient of V between nodes is the multilinear interpolation of central
differences of the node values, clamped to the grid box.  The 4-D
trajectories that leave the box in vx, theta or omega (where the grid's
ghost extrapolation, not the model, sets V) are left out of the lower bound.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2101_05916_amd import workloads as W


def solve(P):
    r = O.solve(O.make_dyn(P.kind, P.params), O.make_grid(P.n, P.lo, P.hi), P.l, P.dlo, P.dhi,
                tol=P.tol, band=P.band)
    assert r["status"] == O.OK
    return r["V"].reshape(P.n)


class Field:
    """Multilinear interpolation of node arrays over the grid box (states
    outside it are clamped to it)."""

    def __init__(self, P, arrays):
        self.h = np.array([(P.hi[i] - P.lo[i]) / (P.n[i] - 1) for i in range(len(P.n))])
        self.lo = np.array(P.lo, dtype=float)
        self.n = np.array(P.n)
        self.arrays = arrays

    def __call__(self, X):
        D = len(self.n)
        t = (np.clip(X, self.lo, self.lo + self.h * (self.n - 1)) - self.lo) / self.h
        i = np.clip(np.floor(t).astype(int), 0, self.n - 2)
        f = t - i
        outs = [np.zeros(len(X)) for _ in self.arrays]
        for c in range(1 << D):
            w = np.ones(len(X))
            idx = []
            for a in range(D):
                b = (c >> a) & 1
                w = w * (f[:, a] if b else 1.0 - f[:, a])
                idx.append(i[:, a] + b)
            for o, A in zip(outs, self.arrays):
                o += w * A[tuple(idx)]
        return outs


def gradient_field(P, V):
    return Field(P, np.gradient(V, *W.axes(P.n, P.lo, P.hi)))


def rk4(f, X, dt):
    k1 = f(X)
    k2 = f(X + 0.5 * dt * k1)
    k3 = f(X + 0.5 * dt * k2)
    k4 = f(X + dt * k3)
    return X + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)


# the models, written out from Sec. IV eq. (3) and Sec. V (not the oracle's code)
def f_x4d(X, S, d):
    g, d1, d0, n0 = 9.81, 8.0, 10.0, 10.0
    return np.stack([X[:, 1] + d, g * np.tan(X[:, 2]), -d1 * X[:, 2] + X[:, 3],
                     -d0 * X[:, 2] + n0 * S], axis=1)


def f_z2d(X, u, d):
    return np.stack([X[:, 1], 0.91 * u - 9.81 + d], axis=1)


def l_x4d(X):
    return 4.0 - np.abs(X[:, 0])


def l_z2d(X):
    return np.minimum(X[:, 0] - 0.5, 2.5 - X[:, 0])


# ---------------------------------------------------------------- 4-D

def x4d_rollouts(P, V, X0, policy, T=3.0, dt=1e-3, seed=0):
    """min_t l from X0 under u* and a disturbance policy, and whether each
    trajectory stayed inside the box in vx, theta, omega."""
    G = gradient_field(P, V)
    smax, dbar = P.params[4], P.dhi[0]
    rng = np.random.default_rng(seed)
    lo, hi = np.array(P.lo), np.array(P.hi)
    X = X0.copy()
    lmin = l_x4d(X)
    inbox = np.ones(len(X), bool)
    dsw = rng.choice([-dbar, dbar], size=len(X))
    every = int(round(0.1 / dt))
    for k in range(int(round(T / dt))):
        if policy == "switch" and k % every == 0:
            dsw = rng.choice([-dbar, dbar], size=len(X))

        def f(Y):
            p = G(Y)
            S = np.where(p[3] >= 0, smax, -smax)  # u*: n0 S p_omega largest
            if policy == "adversarial":
                d = np.where(p[0] >= 0, -dbar, dbar)  # d*: p_x d smallest
            elif policy == "plus":
                d = np.full(len(Y), dbar)
            elif policy == "minus":
                d = np.full(len(Y), -dbar)
            else:
                d = dsw
            return f_x4d(Y, S, d)

        X = rk4(f, X, dt)
        lmin = np.minimum(lmin, l_x4d(X))
        inbox &= np.all((X[:, 1:] >= lo[1:]) & (X[:, 1:] <= hi[1:]), axis=1)
    return lmin, inbox


def x4d_starts(P, V, count, seed=3):
    Vi = Field(P, [V])
    rng = np.random.default_rng(seed)
    lo, hi = np.array(P.lo), np.array(P.hi)
    Xs = lo + 0.2 * (hi - lo) + 0.6 * (hi - lo) * rng.random((8 * count, 4))
    safe = Xs[Vi(Xs)[0] >= 0.2][:count]
    Xu = lo + (hi - lo) * rng.random((40 * count, 4))
    Xu[:, 0] = rng.uniform(-3.9, 3.9, len(Xu))
    unsafe = Xu[Vi(Xu)[0] <= -0.2][:count]
    return Vi, safe, unsafe


def test_x4d_rollouts_both_sides_of_the_zero_level():
    """15^4 x-subsystem, bound 0.5, 500 safe and 200 unsafe starts: the safe
    starts keep at least V(x0) under every disturbance policy (measured:
    never below V(x0) by more than 1e-15); the unsafe starts leave the
    constraint set under the adversarial play, ending within 0.11 of V(x0)
    (0.20 at 11^4)."""
    P = W.quad_x4d(15, 0.5)
    V = solve(P)
    Vi, safe, unsafe = x4d_starts(P, V, 500)
    unsafe = unsafe[:200]
    assert len(safe) == 500 and len(unsafe) == 200
    v_safe = Vi(safe)[0]
    for pol in ("adversarial", "plus", "minus", "switch"):
        lmin, ok = x4d_rollouts(P, V, safe, pol)
        assert ok.mean() > 0.6, (pol, ok.mean())
        assert np.all(lmin[ok] >= v_safe[ok] - 1e-3), (pol, float(np.max((v_safe - lmin)[ok])))
    lmin, _ = x4d_rollouts(P, V, unsafe, "adversarial")
    assert np.all(lmin < 0)
    assert np.all(lmin <= Vi(unsafe)[0] + 0.15), float(np.max(lmin - Vi(unsafe)[0]))


# ---------------------------------------------------------------- 2-D

def z2d_bounds(n, count=6, T=2.0, dt=1e-3, lattice=0.05, seed=5):
    """(largest excess of a one-switch bang-bang margin over V(x0), largest
    shortfall of the u*/d* margin below V(x0)) over `count` safe and
    `count` unsafe starts."""
    P = W.quad_z2d(n, 0.5)
    V = solve(P)
    Vi = Field(P, [V])
    G = gradient_field(P, V)
    dbar = P.dhi[0]
    rng = np.random.default_rng(seed)
    X0 = np.stack([rng.uniform(0.6, 2.4, 60 * count), rng.uniform(-3.0, 3.0, 60 * count)], 1)
    v0 = Vi(X0)[0]
    X0 = np.concatenate([X0[v0 > 0.05][:count], X0[v0 < -0.05][:count]])
    v0 = Vi(X0)[0]
    ts = np.arange(0.0, T + 1e-9, lattice)
    seq = np.array([(ua, ub, t) for ua in (7.0, 16.0) for ub in (7.0, 16.0) for t in ts])
    m, s = len(seq), len(X0)
    # every start with every control sequence, and one u* trajectory per start
    X = np.concatenate([np.repeat(X0, m, axis=0), X0])
    ua = np.concatenate([np.tile(seq[:, 0], s), np.full(s, np.nan)])
    ub = np.concatenate([np.tile(seq[:, 1], s), np.full(s, np.nan)])
    tsw = np.concatenate([np.tile(seq[:, 2], s), np.zeros(s)])
    fb = np.isnan(ua)
    lmin = l_z2d(X)
    for k in range(int(round(T / dt))):
        u_open = np.where(k * dt < tsw, ua, ub)

        def f(Y):
            p = G(Y)[1]
            d = np.where(p >= 0, -dbar, dbar)
            u = np.where(fb, np.where(p >= 0, 16.0, 7.0), u_open)
            return f_z2d(Y, u, d)

        X = rk4(f, X, dt)
        lmin = np.minimum(lmin, l_z2d(X))
    best = lmin[:m * s].reshape(s, m).max(axis=1)
    return float(np.max(best - v0)), float(np.max(v0 - lmin[m * s:]))


def test_z2d_bangbang_upper_bound_and_lower_bound():
    """Vertical model, bound 0.5: one-switch bang-bang controls never beat
    V(x0) by more than eps_h (measured 0.016 at 51^2, 0.0023 at 101^2: it
    shrinks with h), and the u*/d* margin is never below V(x0) - 1e-3."""
    up51, low51 = z2d_bounds(51)
    up101, low101 = z2d_bounds(101)
    assert up51 <= 0.05 and up101 <= 0.01
    assert up101 < up51
    assert low51 <= 1e-3 and low101 <= 1e-3
