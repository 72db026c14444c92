"""Pins of the oracle's state-dependent disturbance bounds (paper Sec. II-A:
d ranges over a set D(x) that depends on the state; Sec. II-C: the learned
bound is a confidence interval at each state).

A field gives every node its own box [lower, upper] per disturbance channel,
laid out (channel, lower/upper, node).  Which test pins what:
  constant field == constant box     test_constant_field_is_the_box   (bitwise, all three models)
  per-node use, channel order        test_field_change_is_local, test_di2x2_channels
  LF bounds over D(x)                test_lf_alpha_field_*            hand-derived maxima
  converged V with z-dependent d     test_z2d_linear_field_closed_form  braking curve with a
                                     position-dependent deceleration (closed form below)
  direction of the bound             test_wider_field_smaller_value   comparison principle of
                                     the monotone first-order scheme
  invalid fields                     test_field_rejects_bad_pairs
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


# k u_hi - g and g - k u_lo of the vertical model (0.91 * 16 - 9.81, 9.81 - 0.91 * 7)
A_UP0 = 0.91 * 16.0 - 9.81
A_DN0 = 9.81 - 0.91 * 7.0


def test_constant_field_is_the_box():
    cases = [(W.quad_z2d(21, 0.5), 300), (W.quad_x4d(7, 0.5), 12),
             (W.di2x2(7, perm=(1, 0, 3, 2), dbar=(0.5, 0.3)), 12)]
    for P, steps in cases:
        a = O.solve(od(P), og(P), P.l, P.dlo, P.dhi, tol=P.tol, max_iter=steps)
        b = O.solve(od(P), og(P), P.l, None, None, tol=P.tol, max_iter=steps,
                    dfield=W.constant_field(P))
        assert a["iterations"] == b["iterations"]
        assert np.array_equal(a["V"], b["V"]), P.name
        assert np.array_equal(a["alpha"], b["alpha"])


def test_di2x2_channels():
    """Channel 0 acts on copy a, channel 1 on copy b: a field with channel 0 =
    box A and channel 1 = box B equals the constant solve with (A, B), and
    differs from the one with the channels exchanged."""
    P = W.di2x2(7, perm=(0, 1, 2, 3), dbar=(0.9, 0.1))
    f = W.constant_field(P)
    a = O.solve(od(P), og(P), P.l, P.dlo, P.dhi, tol=P.tol, max_iter=20, dfield=f)
    b = O.solve(od(P), og(P), P.l, P.dlo, P.dhi, tol=P.tol, max_iter=20)
    c = O.solve(od(P), og(P), P.l, P.dlo, P.dhi, tol=P.tol, max_iter=20, dfield=f[::-1].copy())
    assert np.array_equal(a["V"], b["V"])
    assert np.max(np.abs(a["V"] - c["V"])) > 1e-3


@pytest.mark.parametrize("model", ["z2d", "x4d"])
def test_field_change_is_local(model):
    """Widening one node's box changes L(V) at that node only, and can only
    lower it (H takes the min over a larger disturbance set)."""
    rng = np.random.default_rng(3)
    P = W.quad_z2d(15, 0.5) if model == "z2d" else W.quad_x4d(7, 0.5)
    f = W.constant_field(P)
    V = rng.standard_normal(P.size)
    alpha = O.lf_alpha(od(P), og(P), None, None, dfield=f)
    L0 = O.spatial_op(od(P), og(P), None, None, alpha, V, dfield=f)
    for idx in (0, P.size // 2 + 3, P.size - 1):
        g = f.copy()
        g[0, 0, idx] -= 0.7
        g[0, 1, idx] += 0.4
        L1 = O.spatial_op(od(P), og(P), None, None, alpha, V, dfield=g)
        changed = np.nonzero(L1 != L0)[0]
        assert list(changed) in ([idx], []), (idx, changed[:5])
        assert L1[idx] <= L0[idx]
    # and some single-node widening does change its node
    g = f.copy()
    g[0, 0, :] -= 0.7
    g[0, 1, :] += 0.4
    assert np.count_nonzero(O.spatial_op(od(P), og(P), None, None, alpha, V, dfield=g) != L0) > 0


def test_lf_alpha_field_z2d():
    P = W.quad_z2d(41, 0.5)
    f = W.wind_z2d(41)
    a = O.lf_alpha(od(P), og(P), None, None, dfield=f)
    lo, hi = f[0, 0], f[0, 1]
    # |vz| at the box edge; |k u - g + d| over both controls and both bounds
    want_vz = np.max(np.abs(np.stack([-A_DN0 + lo, -A_DN0 + hi, A_UP0 + lo, A_UP0 + hi])))
    assert a[0] == 4.0
    assert a[1] == pytest.approx(want_vz, rel=1e-15)


def test_lf_alpha_field_x4d():
    P = W.quad_x4d(9, 0.5)
    f = W.wind_x4d(9)
    a = O.lf_alpha(od(P), og(P), None, None, dfield=f)
    a0 = O.lf_alpha(od(P), og(P), P.dlo, P.dhi)
    VX = W.mesh(P.n, P.lo, P.hi)[1].ravel()
    want_x = np.max(np.maximum(np.abs(VX + f[0, 0]), np.abs(VX + f[0, 1])))
    assert a[0] == pytest.approx(want_x, rel=1e-15)
    assert np.array_equal(a[1:], a0[1:])  # the disturbance enters x' only


def linear_field(P, a0, a1, b0, b1):
    """d in [a0 + a1 z, b0 + b1 z] at every node of the vertical model."""
    Z = W.mesh(P.n, P.lo, P.hi)[0].ravel()
    return np.stack([a0 + a1 * Z, b0 + b1 * Z])[None]


def closed_form_linear(Z, VZ, a0, a1, b0, b1, zmin=0.5, zmax=2.5):
    """V* of the vertical model for d in [a0 + a1 z, b0 + b1 z].

    Falling (vz <= 0): full thrust against the lowest disturbance gives the
    upward deceleration a(s) = A_UP0 + a0 + a1 s at height s; the vehicle
    stops at the height zs where the work integral of a from zs to z equals
    vz^2 / 2, then hovers (feasible: every bound stays inside [-4.75, 3.44]).
    Along that path the lowest point is zs and the highest the start, so
    V* = min(zs - zmin, zmax - z).  Rising (vz >= 0): least thrust against
    the highest disturbance, deceleration A_DN0 - b0 - b1 s, stop at zt,
    V* = min(z - zmin, zmax - zt).  The integrals are quadratics in the stop
    height; the root taken tends to z as vz -> 0 (written in the
    cancellation-free form 2C / (B + sqrt(B^2 + 2 a C)))."""
    A = A_UP0 + a0
    C = A * Z + 0.5 * a1 * Z * Z - 0.5 * VZ * VZ
    zs = 2.0 * C / (A + np.sqrt(A * A + 2.0 * a1 * C))
    B = A_DN0 - b0
    b = -b1
    Ct = B * Z + 0.5 * b * Z * Z + 0.5 * VZ * VZ
    zt = 2.0 * Ct / (B + np.sqrt(B * B + 2.0 * b * Ct))
    down = np.minimum(zs - zmin, zmax - Z)
    up = np.minimum(Z - zmin, zmax - zt)
    return np.where(VZ <= 0, down, up)


FIELD_LIN = (-0.8, 0.2, 0.2, 0.25)  # lower -0.8 + 0.2 z, upper 0.2 + 0.25 z


def test_closed_form_linear_reduces_to_constant():
    # a1 = b1 = 0 gives the constant-bound braking curves z - vz^2/(2 a)
    Z, VZ = np.meshgrid(np.linspace(0, 3, 7), np.linspace(-4, 4, 9), indexing="ij")
    V = closed_form_linear(Z, VZ, -0.5, 0.0, 0.5, 0.0)
    down = np.minimum(Z - 0.5 - VZ ** 2 / (2 * (A_UP0 - 0.5)), 2.5 - Z)
    up = np.minimum(Z - 0.5, 2.5 - Z - VZ ** 2 / (2 * (A_DN0 - 0.5)))
    assert np.allclose(V, np.where(VZ <= 0, down, up), atol=1e-12)


def test_z2d_linear_field_closed_form():
    P = W.quad_z2d(101, 0.5)
    f = linear_field(P, *FIELD_LIN)
    r = O.solve(od(P), og(P), P.l, None, None, tol=P.tol, dfield=f)
    assert r["status"] == O.OK
    Z, VZ = W.mesh(P.n, P.lo, P.hi)
    Vc = closed_form_linear(Z, VZ, *FIELD_LIN)
    V = r["V"].reshape(P.n)
    inner = np.abs(VZ) < 3.5
    hz = 3 / 100
    mism = ((V >= 0) != (Vc >= 0)) & inner
    assert np.all(np.abs(Vc[mism]) <= 2 * hz + 1e-9)
    assert np.mean(mism) < 0.01
    near = inner & (np.abs(Vc) < 0.5) & (np.abs(VZ) < 3.0)
    assert np.max(np.abs(V - Vc)[near]) < 0.03
    # the pin separates this field from its mean box: the constant bound
    # [-0.5, 0.575] (the field at z = 1.5) misses the curve by over twice
    # the tolerance above
    Vm = closed_form_linear(Z, VZ, -0.5, 0.0, 0.575, 0.0)
    assert np.max(np.abs(Vm - Vc)[near]) > 0.06


def test_z2d_field_transposed_fails_closed_form():
    """The same bounds laid along vz instead of z give another value function;
    the closed-form pin tells them apart (an index or layout slip in the
    field would be caught)."""
    P = W.quad_z2d(61, 0.5)
    f = linear_field(P, *FIELD_LIN).reshape(1, 2, 61, 61).transpose(0, 1, 3, 2).reshape(1, 2, -1)
    r = O.solve(od(P), og(P), P.l, None, None, tol=P.tol, dfield=np.ascontiguousarray(f))
    Z, VZ = W.mesh(P.n, P.lo, P.hi)
    Vc = closed_form_linear(Z, VZ, *FIELD_LIN)
    near = (np.abs(Vc) < 0.5) & (np.abs(VZ) < 3.0)
    assert np.max(np.abs(r["V"].reshape(P.n) - Vc)[near]) > 0.05


@pytest.mark.parametrize("model", ["z2d", "x4d"])
def test_wider_field_smaller_value(model):
    """First-order Lax-Friedrichs with CFL <= 1 is monotone, so with one
    alpha and dt for both runs, a field that contains another pointwise (H
    smaller everywhere) gives values <= the other's after every step."""
    if model == "z2d":
        P, f = W.quad_z2d(31, 0.5), W.wind_z2d(31)
    else:
        P, f = W.quad_x4d(7, 0.5), W.wind_x4d(7)
    wide = f.copy()
    wide[:, 0] -= 0.3
    wide[:, 1] += 0.2
    alpha = O.lf_alpha(od(P), og(P), None, None, dfield=wide)
    dt = O.dt(og(P), alpha)
    Vn = np.array(P.l)
    Vw = np.array(P.l)
    for _ in range(25):
        Vn, _ = O.iterate(od(P), og(P), None, None, alpha, dt, P.l, Vn, order=1, dfield=f)
        Vw, _ = O.iterate(od(P), og(P), None, None, alpha, dt, P.l, Vw, order=1, dfield=wide)
    assert np.all(Vw <= Vn + 1e-12)
    assert np.max(Vn - Vw) > 1e-3


def test_field_rejects_bad_pairs():
    P = W.quad_z2d(9, 0.5)
    for bad in ("swap", "nan", "inf"):
        f = W.constant_field(P)
        if bad == "swap":
            f[0, 0, 5], f[0, 1, 5] = 0.4, -0.4
        elif bad == "nan":
            f[0, 1, 7] = np.nan
        else:
            f[0, 0, 2] = -np.inf
        r = O.solve(od(P), og(P), P.l, None, None, tol=P.tol, dfield=f)
        assert r["status"] == O.EINVAL, bad


def test_iterate_at_field_matches_iterate():
    P = W.quad_x4d(7, 0.5)
    f = W.wind_x4d(7)
    rng = np.random.default_rng(5)
    V = np.minimum(P.l, rng.standard_normal(P.size))
    alpha = O.lf_alpha(od(P), og(P), None, None, dfield=f)
    dt = O.dt(og(P), alpha)
    Vn, _ = O.iterate(od(P), og(P), None, None, alpha, dt, P.l, V, dfield=f)
    for idx in rng.integers(0, P.size, 25):
        v = O.iterate_at(od(P), og(P), None, None, alpha, dt, P.l, V, idx, dfield=f)
        assert v == pytest.approx(Vn[idx], abs=1e-13)
