"""The 10-D near-hover quadcopter as the paper writes it (Sec. IV, eq. (3)),
decomposed (Sec. III-A), on the device against the oracle.

* The x/y-subsystem with the disturbance on the velocity rate
  (HJR_QUAD_X4DV): every tile family that takes it (narrow and wide planes,
  with and without per-node bounds, and the flat tiles of first-order
  derivatives) after a fixed number of steps, FP64 <= 5e-5 and FP32 <= 1e-4;
  one device step at 41^4 at sampled nodes, <= 2e-6.
* The decomposed safety query (hjr_safety_query_decomposed): the value is
  the minimum of the subsystems', each subsystem's gradient and control go
  to its own components; compared with the oracle's decomposed query to the
  query bars (1e-12, controls exactly where decided).
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


# shape, order, per-node bounds, forced flat tiles
CASES = [((9, 9, 9, 9), 2, False, False), ((5, 6, 7, 75), 2, False, False),
         ((9, 9, 9, 9), 2, True, False), ((5, 6, 7, 75), 2, True, False),
         ((9, 9, 9, 9), 1, False, False), ((9, 9, 9, 9), 2, False, True),
         ((9, 9, 9, 9), 1, True, False)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}-o{c[1]}"
                         f"{'-field' if c[2] else ''}{'-flat' if c[3] else ''}")
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_x4dv_families_match_oracle(case, dt):
    hjr = hjr_()
    shape, order, field, flat = case
    P = W.quad_x4dv(shape, 0.3)
    f = W.wind_x4dv(shape) if field else None
    steps = 30
    ref = O.solve(odyn(P), ogrid(P), P.l, P.dlo, P.dhi, tol=P.tol, order=order, max_iter=steps,
                  dfield=f)
    dtype = torch.float64 if dt == "f64" else torch.float32
    V, st = hjr.solve(hjr.Spec.of(P), dev(P.l, dtype), dtype=dtype, order=order, max_iter=steps,
                      flags=hjr.FLAG_FLAT_TILES if flat else 0,
                      dfield=None if f is None else dev(f, dtype))
    torch.cuda.synchronize()
    err = float(np.max(np.abs(V.cpu().numpy().astype(np.float64) - ref["V"])))
    print(f"x4dv {shape} order {order}{' field' if field else ''}{' flat' if flat else ''} {dt}: "
          f"max|dV| {err:.3e}")
    assert st["iterations"] == ref["iterations"] == steps
    assert np.allclose(st["alpha"][:4], ref["alpha"], rtol=1e-6)
    assert err <= (FP64_STEP_TOL if dt == "f64" else 1e-4)


@pytest.mark.parametrize("field", [False, True])
def test_x4dv_fullsize_sampled_step(field):
    hjr = hjr_()
    P = W.quad_x4dv(41, 0.3)
    f = W.wind_x4dv(41) if field else None
    f32 = None if f is None else f.astype(np.float32).astype(np.float64)
    spec = hjr.Spec.of(P)
    l = dev(P.l, torch.float32)
    fd = None if f is None else dev(f, torch.float32)
    k = 15
    Vk, _ = hjr.solve(spec, l, dtype=torch.float32, max_iter=k, dfield=fd)
    Vk1, _ = hjr.solve(spec, l, V0=Vk.clone(), dtype=torch.float32, max_iter=1, dfield=fd)
    torch.cuda.synchronize()
    a = Vk.cpu().numpy().astype(np.float64)
    b = Vk1.cpu().numpy().astype(np.float64)
    g, d = ogrid(P), odyn(P)
    alpha = O.lf_alpha(d, g, P.dlo, P.dhi, dfield=f32)
    dt = O.dt(g, alpha)
    rng = np.random.default_rng(21)
    n = 41
    corners = [np.ravel_multi_index(tuple((n - 1) * ((c >> i) & 1) for i in range(4)), P.n)
               for c in range(16)]
    idx = np.concatenate([corners, rng.integers(0, P.size, 400)])
    worst = max(abs(O.iterate_at(d, g, P.dlo, P.dhi, alpha, dt, P.l, a, int(i), dfield=f32) - b[i])
                for i in idx)
    print(f"x4dv 41^4{' field' if field else ''} sampled single-step max|dV| {worst:.3e}")
    assert worst <= 2e-6


def quad10d_inputs(rng, nx=(9, 9, 9, 9), nz=(51, 51)):
    """Subsystem specs and smooth random values for x, y (10-D model's form)
    and z."""
    Px, Pz = W.quad_x4dv(nx, 0.3), W.quad_z10(nz, 0.3)
    vals = []
    for P in (Px, Px, Pz):
        G = W.mesh(P.n, P.lo, P.hi)
        V = sum(np.sin(0.6 * (a + 1) * G[a] + rng.uniform(0, 3)) for a in range(P.ndim)).ravel()
        vals.append(V + 0.05 * rng.standard_normal(P.size))
    return (Px, Px, Pz), vals


def oracle_subs(Ps, Vs):
    return [dict(dyn=odyn(P), grid=ogrid(P), V=V, state_index=list(si), control_index=c,
                 dlo=P.dlo, dhi=P.dhi)
            for P, V, si, c in zip(Ps, Vs, W.QUAD10D_STATE_INDEX, W.QUAD10D_CONTROL_INDEX)]


def states10(Ps, n, rng):
    lo = np.array(Ps[0].lo + Ps[1].lo + Ps[2].lo)
    hi = np.array(Ps[0].hi + Ps[1].hi + Ps[2].hi)
    X = lo + (hi - lo) * rng.random((n, 10))
    X[0] = lo
    X[1] = hi
    X[2, 9] = hi[9] + 0.5  # z part outside its box
    X[3, 1] = np.nan
    return X


def compare10(q, ref):
    v = q["value"].cpu().numpy()
    act = q["active"].cpu().numpy()
    bad = ~ref["ok"]
    assert np.array_equal(np.isnan(v), bad) and np.all(act[bad] == -1)
    ok = ref["ok"]
    assert np.max(np.abs(v[ok] - ref["value"][ok])) <= 1e-12
    assert np.max(np.abs(q["sub_value"].cpu().numpy()[ok] - ref["sub_value"][ok])) <= 1e-12
    # the active subsystem, wherever the minimum is not a near-tie
    sv = np.sort(ref["sub_value"][ok], axis=1)
    clear = (sv[:, 1] - sv[:, 0]) > 1e-9
    assert np.array_equal(act[ok][clear], ref["active"][ok][clear])
    g = q["grad"].cpu().numpy()[ok]
    assert np.max(np.abs(g - ref["grad"][ok])) <= 1e-11 * max(1.0, np.abs(ref["grad"][ok]).max())
    # controls where the deciding gradient component (omega_x, omega_y, vz) is not ~0
    u = q["u_star"].cpu().numpy()[ok]
    for c, comp in enumerate((3, 7, 9)):
        decided = np.abs(ref["grad"][ok][:, comp]) > 1e-9
        assert np.array_equal(u[decided, c], ref["u"][ok][decided, c])


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_decomposed_query_matches_oracle(dt):
    hjr = hjr_()
    rng = np.random.default_rng(31)
    Ps, Vs = quad10d_inputs(rng)
    dtype = torch.float64 if dt == "f64" else torch.float32
    Vd = [dev(V, dtype) for V in Vs]
    V64 = [v.cpu().numpy().astype(np.float64) for v in Vd]
    X = states10(Ps, 300, rng)
    U = rng.uniform(-1, 1, (len(X), 3))
    subs = [(hjr.Spec.of(P), V, si, c) for P, V, si, c in
            zip(Ps, Vd, W.QUAD10D_STATE_INDEX, W.QUAD10D_CONTROL_INDEX)]
    q = hjr.query_decomposed(subs, torch.tensor(X, device="cuda"),
                             u_perf=torch.tensor(U, device="cuda"), level=0.2)
    torch.cuda.synchronize()
    ref = O.query_decomposed(oracle_subs(Ps, V64), X, level=0.2, U_perf=U)
    compare10(q, ref)
    uo = q["u_out"].cpu().numpy()
    ok = ref["ok"]
    for c in range(3):
        decided = np.abs(ref["grad"][ok][:, (3, 7, 9)[c]]) > 1e-9
        assert np.array_equal(uo[ok][decided, c], ref["u_out"][ok][decided, c])


def test_quad10d_solve_then_query():
    """The paper's decomposition end to end on the device: x, y (21^4) and z
    (51^2) solved in one batch, then 10-D states queried against the three
    results; the oracle's decomposed query on the device's values checks
    200 of them."""
    hjr = hjr_()
    Ps = W.decomposed_quad10d_paper(21, 51)
    ls = [dev(P.l, torch.float32) for P in Ps]
    Vs = [torch.empty_like(l) for l in ls]
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V) for P, l, V in zip(Ps, ls, Vs)]
    r, stats = hjr.solve_batch(probs, max_iter=8000)
    torch.cuda.synchronize()
    assert r == hjr.OK, [s["status"] for s in stats]
    rng = np.random.default_rng(41)
    X = states10(Ps, 4096, rng)
    subs = [(hjr.Spec.of(P), V, si, c) for P, V, si, c in
            zip(Ps, Vs, W.QUAD10D_STATE_INDEX, W.QUAD10D_CONTROL_INDEX)]
    q = hjr.query_decomposed(subs, torch.tensor(X, device="cuda"))
    torch.cuda.synchronize()
    pick = np.concatenate([np.arange(4), rng.choice(np.arange(4, len(X)), 196, replace=False)])
    V64 = [v.cpu().numpy().astype(np.float64) for v in Vs]
    ref = O.query_decomposed(oracle_subs(Ps, V64), X[pick])
    compare10({k: t[pick] for k, t in q.items()}, ref)
    print("10-D solve:", [s["iterations"] for s in stats], [s["status"] for s in stats])
