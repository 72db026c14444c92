"""Benchmark of the HJ-reachability safe-set solve on one MI355X.

Default workload (one "step", --mode mix): the batched mix of 256 independent
subsystem safe-set solves -- a seeded draw (numpy default_rng(0)) of 2-D
vertical-quadcopter problems on 51^2 .. 201^2 and 4-D x-subsystem problems
on 31^4 .. 61^4 (121 of them, 6.5e8 nodes, 7.8 GB of FP32 V, Vhat and l),
disturbance bounds uniform in [0.2, 1.0], every one solved from a cold start
to convergence (tol 1e-4; the 4-D ones over the residual band |V| < 0.5) in
one batched device solve: captured chunk graphs, autotuned tile heights.
Every step runs the whole path: level set-up, initialisation, both RK stages,
the residual reduction and stop test, and the decomposed batch.

Metric: grid cell-updates per second (nodes x RK2 steps summed over the 256
problems, divided by the wall time of the timed steps).  The JSON line also
carries p50/p99 of the batch latency, safe-set updates/s, the HBM roofline of
the dominant kernel (RK stage 2 of the 4-D family, timed with HIP events on
the engine's stream in a separate pass over the 121 4-D problems, all live,
7.8 GB streamed from HBM each stage) and the oracle's rate on every host
core it may use, on a bounded sample of the same problems.

Other modes (not the headline line): --mode step (the decomposed near-hover
quadcopter's initial safe set: x, y 21^4 -> 41^4 and z 51^2 -> 101^2 in one
batched solve), --mode batch (the same 256 solves, plain one-solve-per-call
vs batched), --mode serve (Poisson request stream through the continuous-
batching server), --mode warm (warm start and coarse-to-fine vs cold on the
4-D x-subsystem), --mode field (the decomposed solve with state-dependent
disturbance bounds, a per-node interval on every grid level, and the roofline
of its stage-2 kernel), --mode query (safety queries -- value, gradient,
optimal control, filter -- on the converged 41^4 x-subsystem: latency per
call and queries/s), --mode quad10d (the 10-D model as the paper writes it:
initial safe set, then a GP-bound update warm-started from the restricted
previous value, coarse to fine, and 10-D decomposed queries on the result),
--mode local (a warm update of the 41^4 x-subsystem computed over the whole
grid and over the band of the previous value only), --mode precision (FP32
and FP64 device results against the oracle's stored values).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="mix",
                    choices=["mix", "mix_kernels", "step", "batch", "serve", "warm", "copy",
                             "precision", "kernels", "field", "field_kernels", "query", "quad10d",
                             "local"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="mix mode: oracle processes (0 = the host cores this process may "
                         "use, at most 16)")
    ap.add_argument("--profile-steps", type=int, default=128,
                    help="mix mode: RK2 steps of the profiled 4-D pass")
    ap.add_argument("--copy-mib", type=int, default=2048, help="copy mode: MiB per copy")
    ap.add_argument("--chunk", type=int, default=None, help="RK2 steps per chunk (default: autotuned)")
    ap.add_argument("--local-n", type=int, default=41, help="local mode: nodes per axis of the 4-D grid")
    ap.add_argument("--local-dbar", type=float, default=0.55, help="local mode: the updated bound")
    ap.add_argument("--walk", type=int, default=0,
                    help="4-D narrow-plane problems: axis-0 planes per walking workgroup "
                         "(0 or -1 = plane tiles, the default)")
    ap.add_argument("--levels", type=int, default=2, help="1 = cold fine grid only")
    ap.add_argument("--count", type=int, default=256, help="batch mode: problems")
    ap.add_argument("--requests", type=int, default=3000, help="serve mode: requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serve mode: req/s")
    ap.add_argument("--hbm-budget-mib", type=int, default=8192,
                    help="serve mode: device-memory budget of the server (MiB)")
    return ap.parse_args()


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


# ---------------------------------------------------------------------------
# mix (default): 256 independent subsystem solves in one batched solve
# ---------------------------------------------------------------------------

def host_cpu():
    """CPU model and core counts of the host this process runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(model=model, nproc=os.cpu_count(), usable=usable)


def _oracle_worker(job):
    """One oracle process: RK2 steps of one problem of the mix from its cold
    start, single thread, until `seconds` have passed (at least one step)."""
    entry, seconds = job
    from oracle import oracle as O
    from paper_2101_05916_amd import workloads as W
    P = W.problem_from_manifest(entry)
    g = O.make_grid(P.n, P.lo, P.hi)
    d = O.make_dyn(P.kind, P.params)
    alpha = O.lf_alpha(d, g, P.dlo, P.dhi)
    dt = O.dt(g, alpha)
    V = P.l.copy()
    t0 = time.perf_counter()
    steps = 0
    while True:
        V, _ = O.iterate(d, g, P.dlo, P.dhi, alpha, dt, P.l, V)
        steps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    return P.size * steps, steps, time.perf_counter() - t0, entry["n"]


def mix_cpu_baseline(seconds, workers, W, count):
    """The oracle as it stands on a bounded sample of the mix: one process per
    usable host core (at most 16), each running RK2 steps of one 4-D problem
    of the mix (the first `workers` of them, in manifest order) for
    `seconds`.  Runs before this process touches the GPU (the workers are
    forked)."""
    import multiprocessing as mp
    cpu = host_cpu()
    n = workers if workers > 0 else min(16, cpu["usable"] or 1)
    man = [e for e in W.batch_manifest(count, seed=0) if e["kind"] == W.QUAD_X4D][:n]
    n = len(man)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(n) as pool:
        res = pool.map(_oracle_worker, [(e, seconds) for e in man])
    wall = time.perf_counter() - t0
    rates = [r[0] / r[2] for r in res]
    # the processes run side by side: their rates add up
    return dict(value=float(sum(rates)), unit="cell-updates/s", cores=n, kind="oracle",
                sample=f"RK2 steps of the first {n} 4-D problems of the mix (sizes "
                       f"{sorted(r[3] for r in res)}^4), one single-threaded FP64 oracle "
                       f"process each, {sum(r[1] for r in res)} steps, "
                       f"{min(r[2] for r in res):.1f}-{max(r[2] for r in res):.1f} s each, "
                       f"{wall:.1f} s wall; value = sum of the process rates",
                per_core=float(np.mean(rates)), cpu_model=cpu["model"], nproc=cpu["nproc"],
                usable_cores=cpu["usable"])


def build_mix(torch, hjr, W, count, only_4d=False):
    """Device inputs of the mix: per problem its spec, l (FP32) and output V."""
    out = []
    for e in W.batch_manifest(count, seed=0):
        if only_4d and e["kind"] != W.QUAD_X4D:
            continue
        P = W.problem_from_manifest(e)
        l = torch.tensor(P.l, dtype=torch.float32, device="cuda")
        out.append((hjr.Spec.of(P), l, torch.empty_like(l)))
        P.l = None
    return out


def mix_problems(hjr, mix):
    return [hjr.make_problem(spec, l, V) for spec, l, V in mix]


def profile_mix_4d(torch, hjr, W, count, chunk, steps, walk=0):
    """Device time per launch of the dominant kernel, RK stage 2 of the 4-D
    family, with HIP events on the engine's stream (HJR_FLAG_PROFILE: the
    stage launches of one chunk in eight, stamped at the kernels' own start
    and end): the mix's 121 4-D problems batched, their first `steps` RK2
    steps from the cold start, during which every one of them is live."""
    mix = build_mix(torch, hjr, W, count, only_4d=True)
    probs = mix_problems(hjr, mix)
    hjr.solve_batch(probs, dtype=torch.float32, max_iter=16, chunk=chunk, walk=walk)
    _, stats = hjr.solve_batch(probs, dtype=torch.float32, max_iter=steps, chunk=chunk,
                               flags=hjr.FLAG_PROFILE, walk=walk)
    s = stats[0]
    nodes = sum(spec.size for spec, _, _ in mix)
    del probs, mix
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return (np.asarray(s["kernel_ms"]), np.asarray(s["kernel_launches"]),
            s["kernel_cell_updates"], nodes)


def mode_mix(args, torch, hjr, W):
    mix = build_mix(torch, hjr, W, args.count)
    n4 = sum(1 for spec, _, _ in mix if len(spec.n) == 4)
    nodes = sum(spec.size for spec, _, _ in mix)
    progress(f"mix: {len(mix)} problems ({n4} 4-D), {nodes:.3e} nodes")
    probs = mix_problems(hjr, mix)

    def run():
        r, stats = hjr.solve_batch(probs, dtype=torch.float32, chunk=args.chunk,
                                   walk=args.walk)
        if r != hjr.OK:
            raise RuntimeError(f"the mix did not converge: {[s['status'] for s in stats]}")
        return stats

    for i in range(args.warmup):
        s0 = time.perf_counter()
        run()
        progress(f"warm-up step {i + 1}/{args.warmup}: {time.perf_counter() - s0:.2f} s")
    torch.cuda.synchronize()
    lat, cu, its = [], 0, None
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        stats = run()
        lat.append((time.perf_counter() - s0) * 1e3)
        cu += sum(s["cell_updates"] for s in stats)
        its = [s["iterations"] for s in stats]
        progress(f"timed step {i + 1}/{args.steps}: {lat[-1] / 1e3:.2f} s")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    del probs, mix
    torch.cuda.empty_cache()
    # dominant kernel: RK stage 2 of the 4-D family reads Vhat, V, l and
    # writes V (4 x 4 B per cell-update); stage 1 reads V and writes Vhat (8 B)
    kms, kn, kcu, n4nodes = profile_mix_4d(torch, hjr, W, args.count, args.chunk,
                                           args.profile_steps, args.walk)
    progress(f"profiled pass: stage 1 {kms[0] / max(kn[0], 1) * 1e3:.1f} us, stage 2 "
             f"{kms[1] / max(kn[1], 1) * 1e3:.1f} us per launch over {n4nodes:.3e} nodes")
    achieved = kcu * 16.0 / (kms[1] * 1e-3) / 1e9
    value = cu / el if el > 0 else 0.0
    out = {
        "metric": "grid cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / max(args.steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batched mix of {args.count} independent subsystem safe-set solves "
                        "(seed 0): 2-D vertical quadcopter 51^2..201^2 and 4-D x-subsystem "
                        "31^4..61^4 (p = 1/2 each), dbar ~ U[0.2, 1.0], cold starts, ENO2+LF+"
                        "TVD-RK2, CFL 0.8, tol 1e-4 (4-D: residual band |V| < 0.5), FP32 "
                        "values / FP64 residual, one batched solve per step",
            "problems": args.count,
            "problems_4d": n4,
            "nodes": nodes,
            "cell_updates_per_step": cu / max(args.steps, 1),
            "iterations_min_max": [min(its), max(its)] if its else None,
        },
        "updates_per_s": args.count * args.steps / el if el > 0 else 0.0,
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "hbm_frac_end_to_end": value * 24.0 / (HBM_PEAK_GBS * 1e9),
        "roofline": {
            "bound": "hbm",
            "kernel": "k_stage<float,2,3,true> (4-D narrow-plane ENO2 family, the deep-pipelined "
                      "kernel of runs of tiles: RK stage 2 + projection + residual), "
                      f"the mix's {n4} 4-D problems batched ({n4nodes} nodes, all live)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("mix_stage2", MIX_TRAFFIC_FILE),
            "bytes_per_cell_update": 16,
            "avg_launch_us": kms[1] / max(kn[1], 1) * 1e3,
            "launches_timed": int(kn[1]),
            "cell_updates_timed": int(kcu),
            "stage1_avg_launch_us": kms[0] / max(kn[0], 1) * 1e3,
            "stage1_plus_stage2_GBs": kcu * 24.0 / ((kms[0] + kms[1]) * 1e-3) / 1e9,
        },
    }
    if getattr(args, "cpu_result", None) is not None:
        out["cpu_baseline"] = args.cpu_result
    return out


def mode_mix_kernels(args, torch, hjr, W):
    """Only the profiled pass of mix mode (the 121 4-D problems, their first
    --profile-steps RK2 steps), for kernel traces and counter collection."""
    kms, kn, kcu, n4nodes = profile_mix_4d(torch, hjr, W, args.count, args.chunk,
                                           args.profile_steps, args.walk)
    return {"mode": "mix_kernels", "walk": args.walk, "nodes": n4nodes, "steps": args.profile_steps,
            "stage_avg_launch_us": [float(kms[i] / max(kn[i], 1) * 1e3) for i in (0, 1)],
            "launches_timed": [int(x) for x in kn], "cell_updates_timed": int(kcu)}


# ---------------------------------------------------------------------------
# headline step
# ---------------------------------------------------------------------------

def build_step(torch, hjr, W, levels):
    """Device inputs of the decomposed quadcopter: per subsystem a list of
    (n, l, V) levels, coarse to fine."""
    subs = [("x", W.quad_x4d, [21, 41]), ("y", W.quad_x4d, [21, 41]), ("z", W.quad_z2d, [51, 101])]
    jobs = []
    for name, mk, ns in subs:
        ns = ns[-levels:]
        lv = []
        for n in ns:
            P = mk(n, 0.5, name)
            l = torch.tensor(P.l, dtype=torch.float32, device="cuda")
            V = torch.empty_like(l)
            lv.append((P.n, l, V))
        spec = hjr.Spec.of(mk(ns[-1], 0.5, name))
        jobs.append((name, spec, lv))
    return jobs


def run_step(hjr, torch, jobs, flags, chunk):
    probs = [hjr.make_problem(spec, None, None, levels=lv) for _, spec, lv in jobs]
    r, stats = hjr.solve_batch(probs, dtype=torch.float32, flags=flags, chunk=chunk)
    return r, stats


def cpu_baseline(seconds, W):
    """The oracle as it stands, on a bounded sample of the workload: RK2
    steps of the 41^4 x-subsystem from its cold start, single thread."""
    from oracle import oracle as O
    P = W.quad_x4d(41, 0.5)
    g = O.make_grid(P.n, P.lo, P.hi)
    d = O.make_dyn(P.kind, P.params)
    alpha = O.lf_alpha(d, g, P.dlo, P.dhi)
    dt = O.dt(g, alpha)
    V = P.l.copy()
    t0 = time.perf_counter()
    steps = 0
    while True:
        V, _ = O.iterate(d, g, P.dlo, P.dhi, alpha, dt, P.l, V)
        steps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    return dict(value=P.size * steps / el, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"{steps} RK2 steps of the 41^4 x-subsystem (FP64 oracle, 1 thread, "
                       f"{el:.1f} s)")


def profile_dominant(torch, hjr, W, chunk, steps=512):
    """Device time per launch of the dominant kernel, measured with HIP
    events on the engine's stream (HJR_FLAG_PROFILE times the stage launches
    of one chunk in eight, the events stamped at each kernel's own start and
    end): the step's two 4-D subsystems on their fine 41^4 grid, batched as
    in the step, for a fixed number of RK2 steps."""
    Ps = [W.quad_x4d(41, 0.5, "x"), W.quad_x4d(41, 0.5, "y")]
    ls = [torch.tensor(P.l, dtype=torch.float32, device="cuda") for P in Ps]
    Vs = [torch.empty_like(l) for l in ls]
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V) for P, l, V in zip(Ps, ls, Vs)]
    hjr.solve_batch(probs, dtype=torch.float32, max_iter=32, chunk=chunk)
    _, stats = hjr.solve_batch(probs, dtype=torch.float32, max_iter=steps, chunk=chunk,
                               flags=hjr.FLAG_PROFILE)
    s = stats[0]
    return np.asarray(s["kernel_ms"]), np.asarray(s["kernel_launches"]), s["kernel_cell_updates"]


def mode_step(args, torch, hjr, W):
    jobs = build_step(torch, hjr, W, args.levels)
    for _ in range(args.warmup):
        run_step(hjr, torch, jobs, 0, args.chunk)
    torch.cuda.synchronize()
    lat = []
    cu = 0
    it_levels = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        r, stats = run_step(hjr, torch, jobs, 0, args.chunk)
        lat.append((time.perf_counter() - s0) * 1e3)
        if r != hjr.OK:
            raise RuntimeError(f"solve did not converge: {stats}")
        cu += sum(s["cell_updates"] for s in stats)
        it_levels = {name: s["level_iterations"][: len(lv)] for (name, _, lv), s in zip(jobs, stats)}
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = cu / el
    cu_step = cu / args.steps
    # dominant kernel: RK stage 2 of the 4-D subsystems reads Vhat, V, l and
    # writes V (4 x 4 B per cell-update); stage 1 reads V and writes Vhat (8 B)
    kms, kn, kcu = profile_dominant(torch, hjr, W, args.chunk)
    achieved = kcu * 16.0 / (kms[1] * 1e-3) / 1e9
    st12 = kcu * 24.0 / ((kms[0] + kms[1]) * 1e-3) / 1e9
    out = {
        "metric": "grid cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "decomposed 10-D near-hover quadcopter, initial safe set: x,y 4-D 41^4 "
                        "+ z 2-D 101^2, FP32 values / FP64 residual, dbar=0.5, ENO2+LF+TVD-RK2, "
                        "CFL 0.8, tol 1e-4, " +
                        ("coarse-to-fine from 21^4 / 51^2, " if args.levels == 2 else "cold fine grid, ") +
                        "3 subsystems in one batched solve",
            "cell_updates_per_step": cu_step,
            "iterations_per_level": it_levels,
        },
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_stage<float,2,3,false> (4-D narrow-plane ENO2 family: RK stage 2 + "
                      "projection + residual), "
                      "x,y 41^4 batched",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("stage2"),
            "bytes_per_cell_update": 16,
            "avg_launch_us": kms[1] / max(kn[1], 1) * 1e3,
            "launches_timed": int(kn[1]),
            "cell_updates_timed": int(kcu),
            "stage1_plus_stage2_GBs": st12,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, W)
    return out


# ---------------------------------------------------------------------------
# field mode: state-dependent disturbance bounds (d in D(x), a GP-shaped
# interval per node) on every level of the decomposed solve
# ---------------------------------------------------------------------------

def field_of(W, kind, n):
    return W.wind_x4d(n) if kind == W.QUAD_X4D else W.wind_z2d(n)


def build_field_step(torch, hjr, W):
    """(name, spec, levels, fields) per subsystem: x, y on 21^4 -> 41^4 with
    the 4-D update band, z on 51^2 -> 101^2, each level with its own field."""
    subs = [("x", W.quad_x4d, [21, 41]), ("y", W.quad_x4d, [21, 41]), ("z", W.quad_z2d, [51, 101])]
    jobs = []
    for name, mk, ns in subs:
        lv, fs = [], []
        for n in ns:
            P = mk(n, 0.5, name)
            l = torch.tensor(P.l, dtype=torch.float32, device="cuda")
            lv.append((P.n, l, torch.empty_like(l)))
            fs.append(torch.tensor(field_of(W, P.kind, n), dtype=torch.float32, device="cuda"))
        P = mk(ns[-1], 0.5, name)
        if P.kind == W.QUAD_X4D:
            P.band = W.BAND_4D_UPDATE
        jobs.append((name, hjr.Spec.of(P), lv, fs))
    return jobs


def field_cpu_baseline(seconds, W):
    """The oracle on a bounded sample of the field workload: RK2 steps of
    the 41^4 x-subsystem with its per-node bounds, single thread."""
    from oracle import oracle as O
    P = W.quad_x4d(41, 0.5)
    f = W.wind_x4d(41)
    g = O.make_grid(P.n, P.lo, P.hi)
    d = O.make_dyn(P.kind, P.params)
    alpha = O.lf_alpha(d, g, None, None, dfield=f)
    dt = O.dt(g, alpha)
    V = P.l.copy()
    t0 = time.perf_counter()
    steps = 0
    while True:
        V, _ = O.iterate(d, g, None, None, alpha, dt, P.l, V, dfield=f)
        steps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    return dict(value=P.size * steps / el, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"{steps} RK2 steps of the 41^4 x-subsystem with per-node bounds "
                       f"(FP64 oracle, 1 thread, {el:.1f} s)")


def field_x4d_problems(torch, hjr, W):
    Ps = [W.quad_x4d(41, 0.5, "x"), W.quad_x4d(41, 0.5, "y")]
    ls = [torch.tensor(P.l, dtype=torch.float32, device="cuda") for P in Ps]
    fs = [torch.tensor(W.wind_x4d(41), dtype=torch.float32, device="cuda") for _ in Ps]
    Vs = [torch.empty_like(l) for l in ls]
    keep = (ls, fs, Vs)
    return [hjr.make_problem(hjr.Spec.of(P), l, V, dfields=[f])
            for P, l, V, f in zip(Ps, ls, Vs, fs)], keep


def mode_field(args, torch, hjr, W):
    jobs = build_field_step(torch, hjr, W)

    def run():
        probs = [hjr.make_problem(spec, None, None, levels=lv, dfields=fs)
                 for _, spec, lv, fs in jobs]
        return hjr.solve_batch(probs, dtype=torch.float32, chunk=args.chunk)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    lat, cu, it_levels, status = [], 0, None, None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        r, stats = run()
        lat.append((time.perf_counter() - s0) * 1e3)
        status = [s["status"] for s in stats]
        cu += sum(s["cell_updates"] for s in stats)
        it_levels = {name: s["level_iterations"][: len(lv)]
                     for (name, _, lv, _), s in zip(jobs, stats)}
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # stage-2 kernel of the 4-D field family: reads Vhat, V, l and the two
    # bounds, writes V (6 x 4 B per cell-update); stage 1 reads V and the
    # bounds and writes Vhat (16 B)
    probs, keep = field_x4d_problems(torch, hjr, W)
    hjr.solve_batch(probs, dtype=torch.float32, max_iter=32, chunk=args.chunk)
    _, st = hjr.solve_batch(probs, dtype=torch.float32, max_iter=512, chunk=args.chunk,
                            flags=hjr.FLAG_PROFILE)
    kms = np.asarray(st[0]["kernel_ms"])
    kn = np.asarray(st[0]["kernel_launches"])
    kcu = st[0]["kernel_cell_updates"]
    achieved = kcu * 24.0 / (kms[1] * 1e-3) / 1e9
    out = {
        "metric": "grid cell-updates/s",
        "value": cu / el,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "decomposed 10-D near-hover quadcopter with state-dependent disturbance "
                        "bounds (GP-shaped mean -/+ 3 sigma per node): x,y 4-D 21^4 -> 41^4 "
                        "(residual band 0.5) + z 2-D 51^2 -> 101^2, FP32 values / FP64 "
                        "residual, ENO2+LF+TVD-RK2, CFL 0.8, tol 1e-4, 3 subsystems in one "
                        "batched solve",
            "cell_updates_per_step": cu / args.steps,
            "iterations_per_level": it_levels,
            "status": status,
        },
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_stage<float,2,X4D narrow, per-node bounds> (RK stage 2 + projection + "
                      "residual), x,y 41^4 batched",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("field_stage2"),
            "bytes_per_cell_update": 24,
            "avg_launch_us": kms[1] / max(kn[1], 1) * 1e3,
            "launches_timed": int(kn[1]),
            "cell_updates_timed": int(kcu),
            "stage1_plus_stage2_GBs": kcu * 40.0 / ((kms[0] + kms[1]) * 1e-3) / 1e9,
        },
    }
    del keep
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = field_cpu_baseline(args.cpu_seconds, W)
    return out


def mode_field_kernels(args, torch, hjr, W):
    """64 RK2 steps of the field workload's x, y on 41^4, launched kernel by
    kernel, for counter collection."""
    probs, keep = field_x4d_problems(torch, hjr, W)
    _, st = hjr.solve_batch(probs, dtype=torch.float32, max_iter=64, chunk=16,
                            flags=hjr.FLAG_NO_GRAPH | hjr.FLAG_NO_PIPELINE)
    torch.cuda.synchronize()
    del keep
    return {"mode": "field_kernels", "workload": "x, y 41^4 FP32 with per-node bounds, batched, "
            "64 RK2 steps", "iterations": st[0]["iterations"]}


# ---------------------------------------------------------------------------
# query mode: safety queries on a converged value function
# ---------------------------------------------------------------------------

def mode_query(args, torch, hjr, W):
    """The 41^4 x-subsystem solved cold on the device (FP32), then safety
    queries (value, gradient, u*, filtered control) at seeded random states:
    per batch size, the wall latency of a call (enqueue + synchronise) and
    the device time per call from HIP events."""
    P = W.quad_x4d(41, 0.5, "x")
    spec = hjr.Spec.of(P)
    V, st = hjr.solve(spec, torch.tensor(P.l, dtype=torch.float32, device="cuda"))
    rng = np.random.default_rng(5)
    lo, hi = np.array(P.lo), np.array(P.hi)
    rows = []
    for n in (1, 64, 4096, 262144, 4194304):
        X = torch.tensor(lo + (hi - lo) * rng.random((n, 4)), device="cuda")
        up = torch.tensor(rng.uniform(-0.3, 0.3, (n, 1)), device="cuda")
        out = hjr.query(spec, V, X, u_perf=up)
        reps = 200 if n <= 4096 else 20
        for _ in range(3):
            hjr.query(spec, V, X, u_perf=up, out=out)
        torch.cuda.synchronize()
        lat = []
        for _ in range(reps):
            t0 = time.perf_counter()
            hjr.query(spec, V, X, u_perf=up, out=out)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            hjr.query(spec, V, X, u_perf=up, out=out)
        e1.record()
        torch.cuda.synchronize()
        dev_ms = e0.elapsed_time(e1) / reps
        rows.append(dict(n=n, p50_ms=pct(lat, 50), p99_ms=pct(lat, 99), device_ms=dev_ms,
                         queries_per_s=n / (dev_ms * 1e-3)))
        progress(f"query n={n}: p50 {rows[-1]['p50_ms']:.3f} ms, device {dev_ms:.4f} ms")
    big = rows[-1]
    # per query: the state (32 B), value, gradient, u*, u_perf and u_out
    # (8 + 32 + 8 + 8 + 8 B), and the 144 distinct FP32 values of the
    # corners' stencils (16 corners and, per axis, two more nodes on each
    # side of the cell: 16 + 4 x 32), which mostly hit in cache
    bpq = 32 + 64 + 144 * 4
    achieved = big["queries_per_s"] * bpq / 1e9
    return {
        "metric": "safety queries/s",
        "value": big["queries_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64 (V stored as f32)",
        "data": "synthetic",
        "config": {"workload": "safety query (value, gradient, u*, least-restrictive filter) on "
                               "the converged 41^4 x-subsystem, uniform random states",
                   "solve_iterations": st["iterations"]},
        "batches": rows,
        "roofline": {"bound": "hbm", "kernel": "k_query<float>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_query": bpq,
                     "avg_launch_us": big["device_ms"] * 1e3, "queries_per_launch": big["n"]},
    }


# ---------------------------------------------------------------------------
# quad10d mode: the 10-D model of the paper, initial safe set and update
# ---------------------------------------------------------------------------

def mode_quad10d(args, torch, hjr, W):
    """x, y (the 10-D model's x-subsystem form, 21^4 -> 41^4, band 0.5) and
    z (51^2 -> 101^2): (1) the initial safe set for the bound +-0.3, cold,
    coarse to fine; (2) the update for GP-shaped per-node bounds (wind near
    a wall for x, y; the vertical wind for z), each level with its own
    field, started on the coarse grid from the previous fine value
    restricted to it; (3) decomposed queries of 10-D states on the updated
    values.  FP32; the 4-D residuals over the band 0.1 (workloads.BAND_X4DV)."""
    levels = {"x": (W.quad_x4dv, [21, 41]), "y": (W.quad_x4dv, [21, 41]),
              "z": (W.quad_z10, [51, 101])}

    def fields_for(name, n):
        if name == "z":
            nn = (n, n)
            Z = W.mesh(nn, W.Z10_BOX[0], W.Z10_BOX[1])[0]
            mu = 1.5 * np.exp(-0.5 * ((Z - 0.6) / 0.3) ** 2)
            return W.gp_bound(mu, 0.1 + 0.05 * np.abs(Z - 1.5))
        return W.wind_x4dv(n)

    jobs = []
    for name, (mk, ns) in levels.items():
        lv, fs = [], []
        for n in ns:
            P = mk(n, 0.3, name)
            l = torch.tensor(P.l, dtype=torch.float32, device="cuda")
            lv.append((P.n, l, torch.empty_like(l)))
            fs.append(torch.tensor(fields_for(name, n), dtype=torch.float32, device="cuda"))
        P = mk(ns[-1], 0.3, name)
        if P.ndim == 4:
            P.band = W.BAND_X4DV
        jobs.append((name, hjr.Spec.of(P), lv, fs, ns))

    def initial():
        probs = [hjr.make_problem(spec, None, None, levels=lv) for _, spec, lv, _, _ in jobs]
        return hjr.solve_batch(probs, dtype=torch.float32, chunk=args.chunk)

    def update(prev):
        probs = []
        for (name, spec, lv, fs, ns), Vfine in zip(jobs, prev):
            V0 = hjr.interp(lv[-1][0], Vfine, lv[0][0], spec.lo, spec.hi)
            lv2 = [(n, l, torch.empty_like(l)) for n, l, _ in lv]
            probs.append((hjr.make_problem(spec, None, None, V0=V0, levels=lv2, dfields=fs), lv2, V0))
        r, st = hjr.solve_batch([p for p, _, _ in probs], dtype=torch.float32, chunk=args.chunk)
        return r, st, [lv2[-1][2] for _, lv2, _ in probs]

    def timed(fn, reps):
        out, ts = None, []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return out, ts

    initial()
    (r0, st0), t_init = timed(initial, args.steps)
    prev = [lv[-1][2].clone() for _, _, lv, _, _ in jobs]
    update(prev)
    (r1, st1, Vnew), t_upd = timed(lambda: update(prev), args.steps)
    cu0 = sum(s["cell_updates"] for s in st0)
    cu1 = sum(s["cell_updates"] for s in st1)
    # 10-D decomposed queries on the updated values
    subs = [(spec, V, si, c) for (_, spec, _, _, _), V, si, c in
            zip(jobs, Vnew, W.QUAD10D_STATE_INDEX, W.QUAD10D_CONTROL_INDEX)]
    lo = np.array(sum((tuple(sp.lo) for _, sp, _, _, _ in jobs), ()))
    hi = np.array(sum((tuple(sp.hi) for _, sp, _, _, _ in jobs), ()))
    rng = np.random.default_rng(10)
    qrows = []
    for n in (1, 4096, 1048576):
        X = torch.tensor(lo + (hi - lo) * rng.random((n, 10)), device="cuda")
        out = hjr.query_decomposed(subs, X)
        lat = []
        for _ in range(50 if n <= 4096 else 10):
            t0 = time.perf_counter()
            hjr.query_decomposed(subs, X, out=out)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
        qrows.append(dict(n=n, p50_ms=pct(lat, 50), p99_ms=pct(lat, 99),
                          queries_per_s=n / (pct(lat, 50) * 1e-3),
                          safe_fraction=float((out["value"] >= 0).float().mean())))
        progress(f"10-D query n={n}: p50 {qrows[-1]['p50_ms']:.3f} ms")
    ms_upd = pct(t_upd, 50)
    return {
        "metric": "grid cell-updates/s",
        "value": cu1 / (ms_upd * 1e-3),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "10-D near-hover quadcopter as the paper writes it (x, y with the "
                               "disturbance on the velocity rate, |S| <= 14 deg; z thrust "
                               "acceleration in [0.6 g, 1.4 g]); safe-set update for GP-shaped "
                               "per-node bounds, warm-started from the restricted previous "
                               "value, 21^4 -> 41^4 (band 0.1) and 51^2 -> 101^2"},
        "initial": {"ms_p50": pct(t_init, 50), "cell_updates": cu0,
                    "iterations_per_level": {j[0]: s["level_iterations"][:2] for j, s in zip(jobs, st0)},
                    "status": [s["status"] for s in st0]},
        "update": {"ms_p50": ms_upd, "ms_p99": pct(t_upd, 99), "cell_updates": cu1,
                   "iterations_per_level": {j[0]: s["level_iterations"][:2] for j, s in zip(jobs, st1)},
                   "status": [s["status"] for s in st1]},
        "query_10d": qrows,
    }


# ---------------------------------------------------------------------------
# local mode: localized warm-start update
# ---------------------------------------------------------------------------

def mode_local(args, torch, hjr, W):
    """x-subsystem on --local-n^4 (41 by default), FP32, residual band 0.5:
    converge for the bound 0.5, then update to --local-dbar (0.55) warm-started from it,
    (a) over the whole grid, (b) over the band of k = 2 and k = 4 cells
    around the previous zero level set only (hjr_solve_local: masked plane
    tiles, tiles without a band node skipped); zero-level disagreement of
    (b) against (a)."""
    n, dbar = args.local_n, args.local_dbar
    P5 = W.quad_x4d(n, 0.5, band=W.BAND_4D_UPDATE)
    P55 = W.quad_x4d(n, dbar, band=W.BAND_4D_UPDATE)
    spec = hjr.Spec.of(P55)
    l = torch.tensor(P5.l, dtype=torch.float32, device="cuda")
    old, _ = hjr.solve(hjr.Spec.of(P5), l)

    def run(fn):
        fn()
        ts = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            V, st = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return V.clone(), dict(ms_p50=pct(ts, 50), iterations=st["iterations"], status=st["status"],
                               cell_updates=st["cell_updates"])

    Vfull, full = run(lambda: hjr.solve(spec, l, V0=old))
    progress(f"local mode full: {full['ms_p50']:.1f} ms, {full['iterations']} steps")
    out = {"mode": "local", "workload": f"x-subsystem {n}^4, FP32, warm update of the bound "
           f"0.5 -> {dbar}", "full": full}
    for k in (2, 4):
        mask, cnt = hjr.band_mask(spec, old, k)
        Vb, row = run(lambda: hjr.solve_local(spec, l, mask, V0=old))
        row.update(band_nodes=cnt, band_fraction=cnt / P55.size,
                   speedup=full["ms_p50"] / row["ms_p50"],
                   zero_level_disagreement=float((Vfull >= 0).ne(Vb >= 0).float().mean()))
        out[f"band_k{k}"] = row
        progress(f"local mode k={k}: {row['ms_p50']:.1f} ms, {row['iterations']} steps")
    return out


# ---------------------------------------------------------------------------
# batch mode: 256 seeded subsystem solves, plain vs batched
# ---------------------------------------------------------------------------

def mode_batch(args, torch, hjr, W):
    man = W.batch_manifest(args.count, seed=0)
    probs, keep = [], []
    for e in man:
        P = W.problem_from_manifest(e)
        l = torch.tensor(P.l, dtype=torch.float32, device="cuda")
        V = torch.empty_like(l)
        keep.append((P, l, V))
    # plain: one solve per call, per-iteration launches, host convergence read
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cu_plain = 0
    for i, (P, l, V) in enumerate(keep):
        _, st = hjr.solve(hjr.Spec.of(P), l, V_out=V, flags=hjr.FLAG_NO_GRAPH | hjr.FLAG_NO_PIPELINE,
                          chunk=1)
        cu_plain += st["cell_updates"]
        if i % 32 == 31:
            progress(f"plain {i + 1}/{len(keep)} solves, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    V_plain = [V.clone() for _, _, V in keep]
    # batched: one engine pass over all problems
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V) for P, l, V in keep]
    t0 = time.perf_counter()
    r, stats = hjr.solve_batch(probs, dtype=torch.float32, chunk=args.chunk)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    cu = sum(s["cell_updates"] for s in stats)
    same = all(torch.equal(a, V) for a, (_, _, V) in zip(V_plain, keep))
    conv = sum(1 for s in stats if s["status"] == 0)
    n4 = sum(1 for P, _, _ in keep if P.ndim == 4)
    return {
        "metric": "safe-set updates/s (batched vs plain)", "mode": "batch",
        "problems": len(keep), "problems_4d": n4, "converged": conv,
        "tol": W.TOL, "band_4d": W.BAND_4D_UPDATE, "dtype": "f32", "data": "synthetic",
        "plain": {"seconds": t_plain, "updates_per_s": len(keep) / t_plain,
                  "cell_updates_per_s": cu_plain / t_plain},
        "batched": {"seconds": t_batch, "updates_per_s": len(keep) / t_batch,
                    "cell_updates_per_s": cu / t_batch},
        "bit_identical": bool(same),
        "speedup": t_plain / t_batch,
    }


# ---------------------------------------------------------------------------
# serve mode: Poisson request stream
# ---------------------------------------------------------------------------

def mode_serve(args, torch, hjr, W):
    insts, reqs = W.serve_stream(args.requests, args.rate, seed=1)
    specs = {}
    ls = {}
    for I in insts:
        P = (W.quad_x4d(I["n"], band=I["band"]) if I["kind"] == W.QUAD_X4D
             else W.quad_z2d(I["n"]))
        specs[I["instance"]] = P
        ls[I["instance"]] = P.l.astype(np.float32)
    srv = hjr.Server(hbm_budget_bytes=args.hbm_budget_mib << 20, max_active=64, chunk=args.chunk or 16)
    seen = set()
    tickets = []
    t0 = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t0
        if r["t"] > now:
            time.sleep(r["t"] - now)
        P = specs[r["instance"]]
        spec = hjr.Spec.of(P)
        spec.dlo, spec.dhi = (-r["dbar"],), (r["dbar"],)
        first = r["instance"] not in seen
        seen.add(r["instance"])
        tickets.append((r, srv.submit(r["instance"], spec, ls[r["instance"]] if first else None)))
    progress(f"submitted {len(tickets)} requests in {time.perf_counter() - t0:.1f} s")
    replies = []
    for i, (r, t) in enumerate(tickets):
        replies.append((r, srv.wait(t)))
        if i % 500 == 499:
            progress(f"{i + 1} replies, {time.perf_counter() - t0:.1f} s")
    wall = time.perf_counter() - t0
    used, budget = srv.memory()
    srv.close()
    warm = [rep for r, rep in replies[200:]]
    lat = [rep["latency_ms"] for rep in warm]
    ok = sum(1 for _, rep in replies if rep["status"] == 0)
    cu = sum(rep["iterations"] * specs[r["instance"]].size for r, rep in replies)
    return {
        "metric": "safe-set updates/s and p50/p99 latency (served)", "mode": "serve",
        "requests": len(replies), "converged": ok, "rate_offered": args.rate,
        "updates_per_s": len(replies) / wall, "cell_updates_per_s": cu / wall,
        # the load the stream asks for: the offered rate times the mean work per request
        "offered_cell_updates_per_s": args.rate * cu / len(replies),
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "mean": float(np.mean(lat))},
        "warm_fraction": float(np.mean([rep["warm"] for rep in warm])),
        "hbm_used_bytes": used, "hbm_budget_bytes": budget, "dtype": "f32", "data": "synthetic",
    }


# ---------------------------------------------------------------------------
# warm-start / coarse-to-fine comparison on the 4-D x-subsystem
# ---------------------------------------------------------------------------

def mode_warm(args, torch, hjr, W):
    """Warm start and coarse-to-fine on the 4-D x-subsystem: the initial
    safe set at dbar 0.5 (21^4 -> 41^4 -> 61^4), then the update to dbar 0.8
    four ways: cold 61^4 (the baseline), cold coarse-to-fine, warm at 61^4
    from the previous value, and the previous value restricted to 21^4,
    warm there, then refined to 41^4 and 61^4."""
    band = W.BAND_4D_UPDATE
    sizes = (21, 41, 61)
    P5 = [W.quad_x4d(n, 0.5, band=band) for n in sizes]
    ls = [torch.tensor(P.l, dtype=torch.float32, device="cuda") for P in P5]
    ns = [P.n for P in P5]
    nodes = [P.size for P in P5]
    spec5 = hjr.Spec.of(P5[-1])
    spec8 = hjr.Spec.of(W.quad_x4d(61, 0.8, band=band))
    mi = 30000
    out = {"metric": "iterations and time: warm / coarse-to-fine vs cold", "mode": "warm",
           "tol": W.TOL, "band": band, "dtype": "f32", "max_iter": mi}

    def rec(name, its, secs, status, V):
        its = [int(i) for i in its]
        cu = sum(i * nodes[len(nodes) - len(its) + k] for k, i in enumerate(its))
        out[name] = {"level_iterations": its, "cell_updates": cu, "seconds": secs,
                     "status": int(status)}
        progress(f"{name}: {its} in {secs:.2f} s")
        return V

    t0 = time.perf_counter()
    Vs, _, _, st = hjr.solve_levels(spec5, ns, ls, max_iter=mi)
    V61 = rec("initial_coarse_to_fine", st["level_iterations"][:3], time.perf_counter() - t0,
              st["status"], Vs[-1])
    t0 = time.perf_counter()
    Vc, s = hjr.solve(spec8, ls[2], max_iter=mi)
    rec("update_cold_61", [s["iterations"]], time.perf_counter() - t0, s["status"], Vc)
    t0 = time.perf_counter()
    Vs1, _, _, s = hjr.solve_levels(spec8, ns, ls, max_iter=mi)
    rec("update_cold_coarse_to_fine", s["level_iterations"][:3], time.perf_counter() - t0,
        s["status"], Vs1[-1])
    t0 = time.perf_counter()
    Vw, s = hjr.solve(spec8, ls[2], V0=V61, max_iter=mi)
    rec("update_warm_61", [s["iterations"]], time.perf_counter() - t0, s["status"], Vw)
    t0 = time.perf_counter()
    V21 = hjr.interp(ns[2], V61, ns[0], P5[2].lo, P5[2].hi)
    Vs2, _, _, s = hjr.solve_levels(spec8, ns, ls, V0=V21, max_iter=mi)
    rec("update_restrict_warm_coarse_to_fine", s["level_iterations"][:3],
        time.perf_counter() - t0, s["status"], Vs2[-1])
    cold = Vc.cpu().numpy() >= 0
    for name, V in (("update_cold_coarse_to_fine", Vs1[-1]), ("update_warm_61", Vw),
                    ("update_restrict_warm_coarse_to_fine", Vs2[-1])):
        out[name]["zero_level_disagreement_vs_cold_61"] = float(
            np.mean((V.cpu().numpy() >= 0) != cold))
    return out


# ---------------------------------------------------------------------------
# precision: the FP32 and FP64 paths against the oracle's stored converged
# values on the configurations' grids
# ---------------------------------------------------------------------------

GOLDEN = os.path.join(ROOT, "tests", "golden")


def precision_cases(W):
    """(label, stored oracle result, problems coarse to fine, warm-start key)
    for every configuration: the files are written by
    tests/golden/make_goldens.py from the FP64 oracle alone."""
    band = W.BAND_4D_UPDATE
    man = W.batch_manifest(256, seed=0)
    z_mix = next(e for e in man if e["kind"] == W.QUAD_Z2D)
    return [
        ("config 1: 2-D vertical quadcopter 101^2, bound 0.5, cold", "z2d_101_d05",
         [W.quad_z2d(101, 0.5, "z")], None),
        ("config 2: x-subsystem 21^4 -> 41^4, bound 0.5", "x4d_chain_d05",
         [W.quad_x4d(n, 0.5, "x") for n in (21, 41)], None),
        ("config 2: z-subsystem 51^2 -> 101^2, bound 0.5", "z2d_chain_d05",
         [W.quad_z2d(n, 0.5, "z") for n in (51, 101)], None),
        ("config 3: x-subsystem 21^4 -> 41^4 -> 61^4, bound 0.5, band 0.5", "x4d_c2f_d05_band",
         [W.quad_x4d(n, 0.5, "x", band=band) for n in (21, 41, 61)], None),
        ("config 3: update to bound 0.8, warm from the 61^4 value on 21^4 -> 41^4 -> 61^4",
         "x4d_upd_d08_band", [W.quad_x4d(n, 0.8, "x", band=band) for n in (21, 41, 61)], "warm21"),
        ("config 4: problem 5 of the mix, 4-D 31^4, band 0.5", "x4d_mix5_31_band",
         [W.problem_from_manifest(man[5])], None),
        (f"config 4: problem {z_mix['index']} of the mix, 2-D {z_mix['n']}^2", "z2d_mix0",
         [W.problem_from_manifest(z_mix)], None),
    ]


def mode_precision(args, torch, hjr, W):
    """FP32 and FP64 device results against the oracle's stored converged
    values, level by level: step counts, max |V - V_oracle| over every stored
    node and over the nodes the stop test covers, and the zero-level
    disagreement (the sign of V against the oracle's FP64 sign at every
    node).  The stored values are the oracle's rounded to float32 (error
    <= 2.4e-7); 41^4 and 61^4 levels of the 61^4 chains are stored at 2^18
    sampled nodes."""
    out = {"metric": "device result vs FP64 oracle", "mode": "precision", "cases": []}
    for label, name, Ps, warm in precision_cases(W):
        with np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False) as z:
            G = {k: z[k] for k in z.files}
        e = {"case": label, "golden": name, "levels": [int(x) for x in G["levels"]],
             "oracle_steps": [int(x) for x in G["level_iterations"]],
             "oracle_seconds": [float(x) for x in G["level_seconds"]]}
        finals = {}
        for dt, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
            ls = [torch.tensor(P.l, dtype=dt, device="cuda") for P in Ps]
            V0 = None if warm is None else torch.tensor(G[warm], dtype=dt, device="cuda")
            # the second of two identical solves is timed (the first builds
            # the engine and captures its graphs)
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Vs, _, _, st = hjr.solve_levels(hjr.Spec.of(Ps[-1]), [P.n for P in Ps], ls, V0=V0,
                                                dtype=dt)
                torch.cuda.synchronize()
                secs = time.perf_counter() - t0
            lv = []
            for k, P in enumerate(Ps):
                V = Vs[k].double().cpu().numpy()
                sign = np.unpackbits(G[f"sign{k}"])[: P.size].astype(bool)
                Vd = V[G[f"idx{k}"]] if f"idx{k}" in G else V
                Vr = G[f"V{k}"].astype(np.float64)
                err = np.abs(Vd - Vr)
                cov = np.abs(Vr) < P.band if P.band > 0 else np.ones(Vr.shape, bool)
                lv.append({"n": int(P.n[0]), "steps": int(st["level_iterations"][k]),
                           "max_abs_err": float(err.max()),
                           "max_abs_err_covered": float(err[cov].max()) if cov.any() else 0.0,
                           "zero_level_disagreement": float(np.mean((V >= 0) != sign)),
                           "sampled": f"idx{k}" in G})
            finals[tag] = Vs[-1].double().cpu().numpy()
            e[tag] = {"status": st["status"], "seconds": secs, "levels": lv}
            del Vs, ls
            torch.cuda.empty_cache()
        e["f32_vs_f64_max_abs_diff"] = float(np.max(np.abs(finals["f32"] - finals["f64"])))
        out["cases"].append(e)
        progress(f"{label}: f32 {[round(x['max_abs_err'], 7) for x in e['f32']['levels']]} "
                 f"f64 {[x['max_abs_err'] for x in e['f64']['levels']]} steps f32 "
                 f"{[x['steps'] for x in e['f32']['levels']]} f64 "
                 f"{[x['steps'] for x in e['f64']['levels']]} oracle {e['oracle_steps']}")
    return out


# ---------------------------------------------------------------------------
# kernels: the dominant kernel's workload alone, for hardware-counter runs
# ---------------------------------------------------------------------------

def mode_kernels(args, torch, hjr, W):
    """64 RK2 steps of the step's two 4-D subsystems on 41^4, batched, launched
    kernel by kernel (no graph), so that a counter collector sees plain
    stage launches of the dominant family."""
    Ps = [W.quad_x4d(41, 0.5, "x"), W.quad_x4d(41, 0.5, "y")]
    ls = [torch.tensor(P.l, dtype=torch.float32, device="cuda") for P in Ps]
    Vs = [torch.empty_like(l) for l in ls]
    probs = [hjr.make_problem(hjr.Spec.of(P), l, V) for P, l, V in zip(Ps, ls, Vs)]
    _, st = hjr.solve_batch(probs, max_iter=64, chunk=16,
                            flags=hjr.FLAG_NO_GRAPH | hjr.FLAG_NO_PIPELINE)
    torch.cuda.synchronize()
    return {"mode": "kernels", "workload": "x, y 41^4 FP32 batched, 64 RK2 steps",
            "iterations": st[0]["iterations"]}


# ---------------------------------------------------------------------------
# copy mode: a plain device copy of known size, to calibrate the HBM byte
# counters (FETCH_SIZE / WRITE_SIZE) that rocprofv3 reports for the kernels
# ---------------------------------------------------------------------------

def mode_copy(args, torch, hjr, W):
    nbytes = args.copy_mib << 20
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(4):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"mode": "copy", "bytes_per_copy": nbytes, "copies": 4}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_stage_decomposed_quad10d.json")
MIX_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_stage_mix256.json")
KERNEL_SOURCES = ["csrc/hjr_stencil.hpp", "csrc/hjr_kernels.hip", "csrc/hjr_device.hpp",
                  "csrc/hjr_engine.cpp", "tuned.json"]


def kernel_hash():
    """Hash of what defines the stage kernels' memory traffic: their sources
    (tile code, launch caps), the engine that sizes their launches and the
    tuned tile heights."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2101_05916_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(stage_key, path=None):
    """HBM bytes per launch from the committed rocprofv3 counters, or None
    when the kernel sources changed since they were taken."""
    try:
        with open(path or TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get(stage_key, {}).get("traffic_bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: each subsystem solve lives on one device "
              "(multi-GPU sharding is not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    from paper_2101_05916_amd import workloads as W
    args.cpu_result = None
    if args.mode == "mix" and not args.no_cpu_baseline:
        # the oracle processes are forked before this process touches the GPU
        progress("oracle baseline on the host cores")
        args.cpu_result = mix_cpu_baseline(args.cpu_seconds, args.cpu_workers, W, args.count)
        progress(f"oracle: {args.cpu_result['value']:.3e} cell-updates/s on "
                 f"{args.cpu_result['cores']} cores")
    import torch
    from paper_2101_05916_amd import hjr
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    hjr.lib()
    fn = {"mix": mode_mix, "mix_kernels": mode_mix_kernels, "step": mode_step, "batch": mode_batch, "serve": mode_serve, "warm": mode_warm,
          "copy": mode_copy, "precision": mode_precision, "kernels": mode_kernels,
          "field": mode_field, "field_kernels": mode_field_kernels, "query": mode_query,
          "quad10d": mode_quad10d, "local": mode_local}[args.mode]
    out = fn(args, torch, hjr, W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
