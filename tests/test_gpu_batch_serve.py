"""Batched, coarse-to-fine and served solves on the device.

Every form must give each problem exactly (bit for bit) what a single
solve of it gives: no arithmetic crosses problems, and the iteration for a
problem is the same sequence of kernels whatever else shares the launch.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2101_05916_amd import workloads as W

from gpu_util import oracle_solve

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


def dev(a, dtype=torch.float32):
    return torch.tensor(np.asarray(a, dtype=np.float64), dtype=dtype, device="cuda")


def single(P, dtype=torch.float32, V0=None, **kw):
    hjr = hjr_()
    V, st = hjr.solve(hjr.Spec.of(P), dev(P.l, dtype), V0=V0, dtype=dtype, **kw)
    torch.cuda.synchronize()
    return V, st


def mixed_problems():
    return [W.quad_x4d(21, 0.5, "x"), W.quad_x4d(17, 0.8, "y", band=0.5),
            W.quad_z2d(101, 0.5, "z"), W.quad_z2d(51, 0.3, "z2"),
            W.quad_x4d((9, 13, 11, 15), 0.6, "r")]


@pytest.mark.parametrize("flags", [0, 1, 2])
def test_batch_bit_identical_to_single(flags):
    hjr = hjr_()
    Ps = mixed_problems()
    ls = [dev(P.l) for P in Ps]
    Vs = [torch.empty_like(l) for l in ls]
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V) for P, l, V in zip(Ps, ls, Vs)]
    r, stats = hjr.solve_batch(probs, flags=flags, max_iter=3000)
    torch.cuda.synchronize()
    for P, V, st in zip(Ps, Vs, stats):
        Vs1, st1 = single(P, max_iter=3000)
        assert st["iterations"] == st1["iterations"], P.name
        assert st["status"] == st1["status"]
        assert torch.equal(V, Vs1), P.name


def test_large_family_runs_capped_and_matches_single():
    """A family whose V, V-hat and l exceed 2 GiB runs FP32 stage 2 with
    fewer workgroups per CU; the kernels stride over tiles, so every
    problem's result equals its single solve bit for bit."""
    hjr = hjr_()
    P = W.quad_x4d(61, 0.5)
    count = 14  # 14 x 61^4 nodes x 12 B = 2.3 GB
    assert count * P.size * 12 > 2 << 30
    l = dev(P.l)
    Vs = [torch.empty_like(l) for _ in range(count)]
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V) for V in Vs]
    r, stats = hjr.solve_batch(probs, max_iter=6, chunk=4)
    torch.cuda.synchronize()
    assert r == hjr.NOT_CONVERGED
    V1, st1 = single(P, max_iter=6, chunk=4)
    for V, st in zip(Vs, stats):
        assert st["iterations"] == st1["iterations"] == 6
        assert torch.equal(V, V1)


def test_batch_stops_each_problem_at_its_own_step():
    hjr = hjr_()
    Ps = [W.quad_z2d(51, 0.5), W.quad_z2d(101, 0.5), W.quad_z2d(101, 0.0)]
    ls = [dev(P.l, torch.float64) for P in Ps]
    Vs = [torch.empty_like(l) for l in ls]
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V) for P, l, V in zip(Ps, ls, Vs)]
    r, stats = hjr.solve_batch(probs, dtype=torch.float64)
    assert r == hjr.OK
    for P, V, st in zip(Ps, Vs, stats):
        ref = oracle_solve(P)
        assert st["iterations"] == ref["iterations"]
        assert np.max(np.abs(V.cpu().numpy() - ref["V"])) <= 5e-5


def test_batch_takes_the_precision_of_its_arrays():
    """FP64 problems solved without a dtype run the FP64 kernels: the same
    step counts and values as with dtype=float64 (once the binding ran the
    FP32 kernels over such buffers), and the oracle's step counts."""
    hjr = hjr_()
    Ps = [W.quad_z2d(51, 0.5), W.quad_x4d(9, 0.5)]
    out = []
    for dtype in (None, torch.float64):
        ls = [dev(P.l, torch.float64) for P in Ps]
        Vs = [torch.empty_like(l) for l in ls]
        probs = [hjr.make_problem(hjr.Spec.of(P), l, V) for P, l, V in zip(Ps, ls, Vs)]
        r, stats = hjr.solve_batch(probs, dtype=dtype, max_iter=20000)
        torch.cuda.synchronize()
        assert r == hjr.OK
        out.append((Vs, stats))
    (Va, sa), (Vb, sb) = out
    for P, a, b, x, y in zip(Ps, Va, Vb, sa, sb):
        assert x["iterations"] == y["iterations"] == oracle_solve(P)["iterations"], P.name
        assert torch.equal(a, b), P.name


def test_batch_not_converged_status():
    hjr = hjr_()
    Ps = [W.quad_z2d(51, 0.5), W.quad_z2d(101, 0.5)]
    ls = [dev(P.l) for P in Ps]
    Vs = [torch.empty_like(l) for l in ls]
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V) for P, l, V in zip(Ps, ls, Vs)]
    r, stats = hjr.solve_batch(probs, max_iter=250)
    assert r == hjr.NOT_CONVERGED
    assert stats[0]["status"] == hjr.OK and stats[0]["iterations"] == 225
    assert stats[1]["status"] == hjr.NOT_CONVERGED and stats[1]["iterations"] == 250


@pytest.mark.parametrize("case", ["2d", "4d"])
def test_levels_equal_manual_composition(case):
    """hjr_solve_levels == solve coarse, hjr_interp with the fine constraint,
    solve fine from that start -- all through the C ABI."""
    hjr = hjr_()
    if case == "2d":
        Pc, Pf = W.quad_z2d(51, 0.5), W.quad_z2d(101, 0.5)
    else:
        Pc, Pf = W.quad_x4d(11, 0.5), W.quad_x4d(21, 0.5)
    lc, lf = dev(Pc.l), dev(Pf.l)
    spec = hjr.Spec.of(Pf)
    Vs, masks, counts, st = hjr.solve_levels(spec, [Pc.n, Pf.n], [lc, lf], masks=True, max_iter=4000)
    Vc, stc = hjr.solve(hjr.Spec.of(Pc), lc, max_iter=4000)
    V0 = hjr.interp(Pc.n, Vc, Pf.n, Pf.lo, Pf.hi, l_dst=lf)
    Vf, stf = hjr.solve(spec, lf, V0=V0, max_iter=4000)
    torch.cuda.synchronize()
    assert torch.equal(Vs[0], Vc) and torch.equal(Vs[1], Vf)
    assert st["level_iterations"][:2] == [stc["iterations"], stf["iterations"]]
    for k, (P, V) in enumerate([(Pc, Vs[0]), (Pf, Vs[1])]):
        m, cnt = hjr.refine_mask(P.n, P.lo, P.hi, V)
        assert torch.equal(masks[k], m) and counts[k] == cnt
        ref, rc = O.refine_mask(O.make_grid(P.n, P.lo, P.hi), V.cpu().numpy().astype(np.float64))
        assert np.array_equal(m.cpu().numpy(), ref) and rc == cnt


def test_levels_fp64_match_oracle_composition():
    hjr = hjr_()
    Pc, Pf = W.quad_z2d(51, 0.5), W.quad_z2d(101, 0.5)
    Vs, _, _, st = hjr.solve_levels(hjr.Spec.of(Pf), [Pc.n, Pf.n],
                                    [dev(Pc.l, torch.float64), dev(Pf.l, torch.float64)])
    rc = oracle_solve(Pc)
    V0 = O.interp(O.make_grid(Pc.n, Pc.lo, Pc.hi), rc["V"], O.make_grid(Pf.n, Pf.lo, Pf.hi))
    rf = oracle_solve(Pf, V0=V0)
    assert st["level_iterations"][:2] == [rc["iterations"], rf["iterations"]]
    assert np.max(np.abs(Vs[1].cpu().numpy() - rf["V"])) <= 5e-5


def test_batch_multilevel_jobs_equal_single_levels():
    hjr = hjr_()
    jobs = [(W.quad_x4d(11, 0.5), W.quad_x4d(21, 0.5)), (W.quad_z2d(51, 0.4), W.quad_z2d(101, 0.4))]
    probs, outs = [], []
    for Pc, Pf in jobs:
        lc, lf = dev(Pc.l), dev(Pf.l)
        Vc, Vf = torch.empty_like(lc), torch.empty_like(lf)
        outs.append((Pc, Pf, lc, lf, Vc, Vf))
        probs.append(hjr.make_problem(hjr.Spec.of(Pf), None, None,
                                      levels=[(Pc.n, lc, Vc), (Pf.n, lf, Vf)]))
    r, stats = hjr.solve_batch(probs, max_iter=4000)
    for (Pc, Pf, lc, lf, Vc, Vf), st in zip(outs, stats):
        Vs, _, _, st1 = hjr.solve_levels(hjr.Spec.of(Pf), [Pc.n, Pf.n], [lc, lf], max_iter=4000)
        assert torch.equal(Vs[0], Vc) and torch.equal(Vs[1], Vf)
        assert st["level_iterations"] == st1["level_iterations"]


def test_batch_large_set_runs_of_tiles_bit_identical():
    """Four 61^4 problems batched hold more plane tiles than 16 per workgroup
    of a capped grid, so the launch gives each workgroup a run of tiles and
    takes the deeper-pipelined FP32 kernels; one 61^4 problem alone runs the
    capped grid.  The arithmetic per node is the same: every result equals
    its single solve bit for bit (30 steps from the cold start)."""
    hjr = hjr_()
    Ps = [W.quad_x4d(61, d, f"p{i}") for i, d in enumerate((0.3, 0.5, 0.7, 0.9))]
    ls = [dev(P.l) for P in Ps]
    Vs = [torch.empty_like(l) for l in ls]
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V) for P, l, V in zip(Ps, ls, Vs)]
    r, stats = hjr.solve_batch(probs, max_iter=30)
    torch.cuda.synchronize()
    for P, l, V, st in zip(Ps, ls, Vs, stats):
        V1, st1 = single(P, max_iter=30)
        assert st["iterations"] == st1["iterations"] == 30
        assert torch.equal(V, V1)


@pytest.mark.parametrize("pair", ["x4d", "z2d"])
def test_batch_per_level_order_matches_oracle(pair):
    """A chain whose coarse level runs the first-order scheme and whose fine
    level runs ENO2 (Sec. III-C: cheap gradient approximations on the coarse
    grid), in FP64: each level against the oracle run
    with that level's order, started the same way (the coarse level cold, the
    fine level from the multilinear interpolation of the coarse result)."""
    hjr = hjr_()
    Pc, Pf = ((W.quad_x4d(11, 0.5), W.quad_x4d(17, 0.5)) if pair == "x4d"
              else (W.quad_z2d(51, 0.4), W.quad_z2d(101, 0.4)))
    lc, lf = dev(Pc.l, torch.float64), dev(Pf.l, torch.float64)
    Vc, Vf = torch.empty_like(lc), torch.empty_like(lf)
    prob = hjr.make_problem(hjr.Spec.of(Pf), None, None,
                            levels=[(Pc.n, lc, Vc), (Pf.n, lf, Vf)], orders=[1, 2])
    r, stats = hjr.solve_batch([prob], max_iter=20000)
    torch.cuda.synchronize()
    rc = oracle_solve(Pc, order=1)
    V0 = O.interp(O.make_grid(Pc.n, Pc.lo, Pc.hi), rc["V"], O.make_grid(Pf.n, Pf.lo, Pf.hi))
    rf = oracle_solve(Pf, V0=V0, order=2)
    assert stats[0]["level_iterations"][:2] == [rc["iterations"], rf["iterations"]]
    assert np.max(np.abs(Vc.cpu().numpy() - rc["V"])) <= 1e-9
    assert np.max(np.abs(Vf.cpu().numpy() - rf["V"])) <= 5e-5  # the FP64 parity bar
    # the coarse level is the plain order-1 solve, bit for bit
    V1, st1 = single(Pc, dtype=torch.float64, order=1)
    assert torch.equal(V1, Vc) and st1["iterations"] == rc["iterations"]


def test_graph_replays_stable():
    """Captured chunk graphs are reused across calls (engine pool); replays
    interleaved with eager work give identical results every time."""
    P = W.quad_z2d(101, 0.5)
    V0, st0 = single(P)
    for _ in range(3):
        x = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        y = (x * 2).sum().item()  # eager work between replays
        V, st = single(P)
        assert st["iterations"] == st0["iterations"]
        assert torch.equal(V, V0)
        assert y == y


def test_in_place_warm_update():
    # V0 may alias V_out
    hjr = hjr_()
    P5, P8 = W.quad_z2d(101, 0.5), W.quad_z2d(101, 0.8)
    V5, _ = single(P5)
    ref, stref = single(P8, V0=V5.clone())
    V = V5.clone()
    out, st = hjr.solve(hjr.Spec.of(P8), dev(P8.l), V0=V, V_out=V)
    assert out.data_ptr() == V.data_ptr()
    assert torch.equal(V, ref) and st["iterations"] == stref["iterations"]


def test_nan_constraint_does_not_converge():
    P = W.quad_z2d(31, 0.5)
    l = P.l.copy()
    l[100] = np.nan
    hjr = hjr_()
    V, st = hjr.solve(hjr.Spec.of(P), dev(l), max_iter=40)
    assert st["status"] == hjr.NOT_CONVERGED and st["iterations"] == 40


# ---------------------------------------------------------------- serving

def server_reference(reqs, specs, ls):
    """Sequential single solves with the same warm-start rule as the server:
    the first request of an instance is cold, later ones start from the
    instance's last converged value."""
    hjr = hjr_()
    last = {}
    out = []
    for inst, dbar in reqs:
        P = specs[inst]
        spec = hjr.Spec.of(P)
        spec.dlo, spec.dhi = (-dbar,), (dbar,)
        V, st = hjr.solve(spec, ls[inst], V0=last.get(inst))
        torch.cuda.synchronize()
        if st["status"] == hjr.OK:
            last[inst] = V
        out.append((V.cpu().numpy(), st["iterations"]))
    return out, last


def make_instances():
    specs = {0: W.quad_z2d(51), 1: W.quad_z2d(101), 2: W.quad_x4d(17),
             3: W.quad_x4d(21, band=W.BAND_4D_UPDATE)}
    return specs, {k: dev(P.l) for k, P in specs.items()}


REQS = [(0, 0.5), (1, 0.5), (2, 0.5), (0, 0.8), (3, 0.4), (1, 0.3), (2, 0.7), (0, 0.6),
        (3, 0.9), (1, 0.7)]


@pytest.mark.parametrize("mode", ["alone", "mix"])
def test_server_matches_sequential_solves(mode):
    """Each result equals the single-solve reference whether the requests
    run one at a time or all overlap on the device (continuous batching).
    One at a time, every reply's value (the instance's resident value right
    after it) is compared with the reference bit for bit; overlapped, a later
    request of an instance may already have replaced it, so the values are
    compared at the end, and an intermediate value is checked through the
    step count and result of the request warm-started from it."""
    hjr = hjr_()
    specs, ls = make_instances()
    ref, last = server_reference(REQS, specs, ls)
    with hjr.Server(max_active=8, chunk=16) as srv:
        seen, tickets, replies = set(), [], []
        for inst, dbar in REQS:
            spec = hjr.Spec.of(specs[inst])
            spec.dlo, spec.dhi = (-dbar,), (dbar,)
            lh = specs[inst].l.astype(np.float32) if inst not in seen else None
            seen.add(inst)
            t = srv.submit(inst, spec, lh)
            if mode == "alone":
                rep = srv.wait(t)
                replies.append(rep)
                rv = ref[len(replies) - 1][0]
                assert rep["status"] == hjr.OK
                assert np.array_equal(srv.read_value(inst, specs[inst].size), rv)
            else:
                tickets.append(t)
        if mode == "mix":
            replies = [srv.wait(t) for t in tickets]
        for (rv, rit), rep in zip(ref, replies):
            assert rep["status"] == hjr.OK
            assert rep["iterations"] == rit
        for inst, V in last.items():
            got = srv.read_value(inst, specs[inst].size)
            assert np.array_equal(got, V.cpu().numpy())
        # warm flags: first request per instance cold, then warm
        firsts = {}
        for (inst, _), rep in zip(REQS, replies):
            assert rep["warm"] == (inst in firsts)
            firsts[inst] = True


def test_server_small_budget_queues_and_evicts():
    """A budget that holds about one 4-D instance at a time: requests wait
    for memory, idle instances are evicted (their next request is cold),
    and every result still equals a single solve with that start."""
    hjr = hjr_()
    P = W.quad_x4d(21)
    N = P.size
    budget = 2 << 20  # tables + one instance + its working set at 21^4 FP32 (~0.8 MB each)
    budget = max(budget, 6 * 4 * N + (1 << 20))
    specs = {k: W.quad_x4d(21) for k in range(3)}
    ls = {k: dev(P.l) for k, P in specs.items()}
    with hjr.Server(hbm_budget_bytes=budget, max_active=4, chunk=16) as srv:
        used, b = srv.memory()
        assert b == budget
        tickets = []
        for k in range(3):
            spec = hjr.Spec.of(specs[k])
            tickets.append(srv.submit(k, spec, specs[k].l.astype(np.float32)))
        reps = [srv.wait(t) for t in tickets]
        used, _ = srv.memory()
        assert used <= budget
        V1, st1 = hjr.solve(hjr.Spec.of(specs[0]), ls[0])
        torch.cuda.synchronize()
        for rep in reps:
            assert rep["status"] == hjr.OK and rep["iterations"] == st1["iterations"]
        # every instance still resident holds exactly the single solve's value
        resident = 0
        for k in range(3):
            try:
                got = srv.read_value(k, N)
            except hjr.HjrError as e:
                assert e.status == hjr.ENOTFOUND
                continue  # evicted to make room for a later instance
            resident += 1
            assert np.array_equal(got, V1.cpu().numpy())
        assert resident >= 1


def test_server_not_converged_keeps_resident_value():
    hjr = hjr_()
    P = W.quad_z2d(51)
    with hjr.Server(max_active=2, chunk=8, max_iter=300) as srv:
        spec = hjr.Spec.of(P)
        rep = srv.wait(srv.submit(7, spec, P.l.astype(np.float32)))
        assert rep["status"] == hjr.OK
        good = srv.read_value(7, P.size)
    with hjr.Server(max_active=2, chunk=8, max_iter=5) as srv:
        rep = srv.wait(srv.submit(7, spec, P.l.astype(np.float32)))
        assert rep["status"] == hjr.NOT_CONVERGED and rep["iterations"] == 5
        with pytest.raises(hjr.HjrError):
            srv.read_value(7, P.size)  # nothing converged yet: no resident value
    assert good.shape == (P.size,)


def test_server_rejects_bad_requests():
    hjr = hjr_()
    P = W.quad_z2d(51)
    with hjr.Server(max_active=2) as srv:
        with pytest.raises(hjr.HjrError):
            srv.submit(1, hjr.Spec.of(P), None)  # first request must bring l
        t = srv.submit(1, hjr.Spec.of(P), P.l.astype(np.float32))
        Q = W.quad_z2d(61)
        with pytest.raises(hjr.HjrError):
            srv.submit(1, hjr.Spec.of(Q), None)  # grid of a known instance changed
        assert srv.wait(t)["status"] == hjr.OK
        with pytest.raises(hjr.HjrError):
            srv.poll(987654)
