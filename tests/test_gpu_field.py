"""Device solves with state-dependent disturbance bounds (paper Sec. II-A: d
ranges over D(x); Sec. II-C: the learned bound is a confidence interval at
every state) against the FP64 oracle on identical seeded inputs.

Bars as for the constant-box parity tests: FP64 max|dV| <= 5e-5 and equal
step counts, FP32 max|dV| <= 1e-4.  Every tile family that takes fields is
covered (narrow and wide planes of both plane models, and the flat tiles:
first-order derivatives, forced flat tiles, the two-channel test model), as
are the multi-level, batched and served forms, invalid fields and a sampled
step at the benchmark size.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2101_05916_amd import workloads as W

from gpu_util import odyn, ogrid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64_TOL = 5e-5
FP64_STEP_TOL = 1e-10  # fixed runs of <= 30 steps: the two evaluation orders agree to rounding


@pytest.fixture(scope="module", autouse=True)
def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_05916_amd import hjr
    hjr.lib()


def hjr_():
    from paper_2101_05916_amd import hjr
    return hjr


def dev(a, dtype):
    return torch.tensor(np.asarray(a, dtype=np.float64), dtype=dtype, device="cuda")


def field_for(P):
    """Synthetic GP-shaped bounds on P's grid (two channels for DI2X2: its
    constant boxes widened by a smooth, node-dependent margin)."""
    if P.kind == W.QUAD_Z2D:
        return W.wind_z2d(P.n)
    if P.kind == W.QUAD_X4D:
        return W.wind_x4d(P.n)
    f = W.constant_field(P)
    u = 0.5 + 0.5 * np.sin(0.37 * np.arange(P.size))
    f[:, 0] -= 0.2 * u
    f[:, 1] += 0.1 * u[::-1]
    return f


def oracle_field(P, f, V0=None, max_iter=100000, order=2, l=None):
    return O.solve(odyn(P), ogrid(P), P.l if l is None else l, None, None, tol=P.tol, V0=V0,
                   order=order, max_iter=max_iter, band=P.band, dfield=f)


def device_field(P, f, dtype, V0=None, max_iter=100000, order=2, flags=0, l=None):
    hjr = hjr_()
    v0 = None if V0 is None else dev(V0, dtype)
    V, st = hjr.solve(hjr.Spec.of(P), dev(P.l if l is None else l, dtype), V0=v0, dtype=dtype,
                      max_iter=max_iter, order=order, flags=flags, dfield=dev(f, dtype))
    torch.cuda.synchronize()
    return V.cpu().numpy().astype(np.float64), st


# model, shape, order, flat-tile flag: one case per family that takes fields
CASES = [("z2d", (51, 51), 2, False), ("z2d", (83, 97), 2, False),
         ("x4d", (9, 9, 9, 9), 2, False), ("x4d", (5, 6, 7, 75), 2, False),
         ("x4d", (9, 9, 9, 9), 1, False), ("z2d", (51, 51), 2, True),
         ("di2x2", (7, 7, 7, 7), 2, False)]


def make(kind, shape):
    if kind == "z2d":
        return W.quad_z2d(shape, 0.5)
    if kind == "x4d":
        return W.quad_x4d(shape, 0.5)
    return W.di2x2(shape[0], perm=(1, 0, 3, 2), dbar=(0.5, 0.3))


@pytest.mark.parametrize("case", CASES,
                         ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[1]))}-o{c[2]}{'-flat' if c[3] else ''}")
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_field_families_match_oracle(case, dt):
    hjr = hjr_()
    kind, shape, order, flat = case
    P = make(kind, shape)
    f = field_for(P)
    steps = 30
    ref = oracle_field(P, f, order=order, max_iter=steps)
    V, st = device_field(P, f, torch.float64 if dt == "f64" else torch.float32, order=order,
                         max_iter=steps, flags=hjr.FLAG_FLAT_TILES if flat else 0)
    err = float(np.max(np.abs(V - ref["V"])))
    print(f"field {kind} {shape} order {order} {dt}{' flat' if flat else ''}: max|dV| {err:.3e}")
    assert st["iterations"] == ref["iterations"] == steps
    assert np.allclose(st["alpha"][:P.ndim], ref["alpha"], rtol=1e-6)
    assert err <= (FP64_STEP_TOL if dt == "f64" else 1e-4)


def test_field_z2d_converged_fp64():
    P = W.quad_z2d(101, 0.5)
    f = W.wind_z2d(101)
    ref = oracle_field(P, f)
    V, st = device_field(P, f, torch.float64)
    assert ref["status"] == O.OK and st["status"] == 0
    assert st["iterations"] == ref["iterations"]
    assert np.max(np.abs(V - ref["V"])) <= FP64_TOL


def test_field_x4d_band_converged_fp64():
    P = W.quad_x4d(15, 0.5, band=W.BAND_4D_UPDATE)
    f = W.wind_x4d(15)
    ref = oracle_field(P, f)
    V, st = device_field(P, f, torch.float64)
    assert ref["status"] == O.OK
    assert st["iterations"] == ref["iterations"]
    assert np.max(np.abs(V - ref["V"])) <= FP64_TOL


def test_field_levels_fp64_match_oracle_composition():
    """Coarse-to-fine with a field per level: level 0 from l, level 1 from
    min(l, interp(V0*)), each with its own grid's bounds."""
    hjr = hjr_()
    P0, P1 = W.quad_z2d(51, 0.5), W.quad_z2d(101, 0.5)
    f0, f1 = W.wind_z2d(51), W.wind_z2d(101)
    r0 = oracle_field(P0, f0)
    V1in = O.interp(ogrid(P0), r0["V"], ogrid(P1))
    r1 = oracle_field(P1, f1, V0=V1in)
    Vs, _, _, st = hjr.solve_levels(hjr.Spec.of(P1), [P0.n, P1.n],
                                    [dev(P0.l, torch.float64), dev(P1.l, torch.float64)],
                                    dtype=torch.float64,
                                    dfields=[dev(f0, torch.float64), dev(f1, torch.float64)])
    torch.cuda.synchronize()
    assert st["level_iterations"][:2] == [r0["iterations"], r1["iterations"]]
    assert np.max(np.abs(Vs[1].cpu().numpy() - r1["V"])) <= FP64_TOL


def test_field_batch_bit_identical_to_single():
    """Problems with and without fields share every launch of a batch; each
    result equals its single solve bit for bit."""
    hjr = hjr_()
    Ps = [W.quad_x4d(13, 0.5, "xf", band=0.5), W.quad_x4d(13, 0.5, "xb", band=0.5),
          W.quad_z2d(51, 0.5, "zf"), W.quad_z2d(61, 0.5, "zb"),
          W.quad_x4d((5, 6, 7, 75), 0.5, "wf")]
    fields = [W.wind_x4d(13), None, W.wind_z2d(51), None, W.wind_x4d((5, 6, 7, 75))]
    dt = torch.float32
    ls = [dev(P.l, dt) for P in Ps]
    fs = [None if f is None else dev(f, dt) for f in fields]
    Vs = [torch.empty_like(l) for l in ls]
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V, dfields=[f])
             for P, l, V, f in zip(Ps, ls, Vs, fs)]
    r, stats = hjr.solve_batch(probs, max_iter=400)
    torch.cuda.synchronize()
    for P, l, V, f, s in zip(Ps, ls, Vs, fs, stats):
        Vref, st = hjr.solve(hjr.Spec.of(P), l, dtype=dt, max_iter=400, dfield=f)
        torch.cuda.synchronize()
        assert s["iterations"] == st["iterations"], P.name
        assert torch.equal(V, Vref), P.name


@pytest.mark.parametrize("bad", ["swap", "nan", "inf"])
def test_invalid_field_rejected(bad):
    hjr = hjr_()
    P = W.quad_z2d(31, 0.5)
    f = W.wind_z2d(31)
    if bad == "swap":
        f[0, 0, 100], f[0, 1, 100] = f[0, 1, 100] + 0.1, f[0, 0, 100]
    elif bad == "nan":
        f[0, 1, 7] = np.nan
    else:
        f[0, 0, 500] = -np.inf
    for dt in (torch.float32, torch.float64):
        out = torch.full((P.size,), 7.0, dtype=dt, device="cuda")
        with pytest.raises(hjr.HjrError) as e:
            hjr.solve(hjr.Spec.of(P), dev(P.l, dt), V_out=out, dtype=dt, dfield=dev(f, dt))
        assert e.value.status == hjr.EINVAL
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())  # nothing was written
        # the batch checks every field before solving anything
        V = torch.full((P.size,), 7.0, dtype=dt, device="cuda")
        Q = W.quad_z2d(31, 0.5)
        W2 = torch.full((Q.size,), 7.0, dtype=dt, device="cuda")
        probs = [hjr.make_problem(hjr.Spec.of(Q), dev(Q.l, dt), W2),
                 hjr.make_problem(hjr.Spec.of(P), dev(P.l, dt), V, dfields=[dev(f, dt)])]
        with pytest.raises(hjr.HjrError) as e:
            hjr.solve_batch(probs, dtype=dt)
        assert e.value.status == hjr.EINVAL
        torch.cuda.synchronize()
        assert bool((W2 == 7.0).all()) and bool((V == 7.0).all())
    # a valid solve right after still works (the pooled engine is intact)
    V, st = device_field(P, W.wind_z2d(31), torch.float32, max_iter=5)
    assert st["iterations"] == 5


def test_server_field_requests_match_single_solves():
    """GP updates as served requests: each request carries its own field;
    the first is cold, the next warm-starts from the resident value, and the
    results equal single solves with the same starts."""
    hjr = hjr_()
    P = W.quad_z2d(51, 0.5)
    fa = W.wind_z2d(51)
    fb = W.wind_z2d(51, peak=2.0, z0=0.6)
    spec = hjr.Spec.of(P)
    l = dev(P.l, torch.float32)
    Va, sa = hjr.solve(spec, l, dfield=dev(fa, torch.float32))
    Vb, sb = hjr.solve(spec, l, V0=Va.clone(), dfield=dev(fb, torch.float32))
    torch.cuda.synchronize()
    with hjr.Server(max_active=4, chunk=16) as srv:
        ra = srv.wait(srv.submit(3, spec, P.l.astype(np.float32), dfield_host=fa))
        rb = srv.wait(srv.submit(3, spec, None, dfield_host=fb))
        assert ra["status"] == rb["status"] == hjr.OK
        assert (ra["warm"], rb["warm"]) == (False, True)
        assert ra["iterations"] == sa["iterations"] and rb["iterations"] == sb["iterations"]
        assert np.array_equal(srv.read_value(3, P.size), Vb.cpu().numpy())
        bad = fa.copy()
        bad[0, 0, 3] = np.nan
        with pytest.raises(hjr.HjrError):
            srv.submit(3, spec, None, dfield_host=bad)


def test_field_x4d_fullsize_sampled_step():
    """41^4 in FP32 with a field (the narrow-plane field family at the
    benchmark size): k device steps, one more, and the last step at sampled
    nodes against the oracle's single-node step from the device's V_k."""
    hjr = hjr_()
    P = W.quad_x4d(41, 0.5)
    f = W.wind_x4d(41)
    f32 = f.astype(np.float32).astype(np.float64)  # the bounds the device holds
    spec = hjr.Spec.of(P)
    l = dev(P.l, torch.float32)
    fd = dev(f, torch.float32)
    k = 15
    Vk, _ = hjr.solve(spec, l, dtype=torch.float32, max_iter=k, dfield=fd)
    Vk1, _ = hjr.solve(spec, l, V0=Vk.clone(), dtype=torch.float32, max_iter=1, dfield=fd)
    torch.cuda.synchronize()
    a = Vk.cpu().numpy().astype(np.float64)
    b = Vk1.cpu().numpy().astype(np.float64)
    g, d = ogrid(P), odyn(P)
    alpha = O.lf_alpha(d, g, None, None, dfield=f32)
    dt = O.dt(g, alpha)
    n = 41
    rng = np.random.default_rng(11)
    corners = [np.ravel_multi_index(tuple((n - 1) * ((c >> i) & 1) for i in range(4)), P.n)
               for c in range(16)]
    idx = np.concatenate([corners, rng.integers(0, P.size, 400)])
    worst = 0.0
    for i in idx:
        v = O.iterate_at(d, g, None, None, alpha, dt, P.l, a, int(i), dfield=f32)
        worst = max(worst, abs(v - b[i]))
    print(f"field x4d 41^4 sampled single-step max|dV| {worst:.3e}")
    assert worst <= 2e-6
