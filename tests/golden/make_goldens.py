"""Write the stored oracle results of converged solves that the GPU parity
tests and bench.py's precision mode compare against (tests/golden/*.npz).

Calls only the FP64 oracle (oracle/) and the seeded input generators
(paper_2101_05916_amd/workloads.py, which hold no solver arithmetic).
Nothing here comes from the device library.

What each case computes (paper Sec. II-A eq. (2): iterate until the value
stops changing; Sec. III-B: warm start; Sec. III-C: converge on a coarse grid,
carry the value to a finer one by multilinear interpolation, continue):

  chain_d05      21^4 cold -> 41^4, bound 0.5, stop over every node: the
                 x- and y-subsystems of the decomposed near-hover quadcopter's
                 initial safe set.
  c2f_d05_band   21^4 cold -> 41^4 -> 61^4, bound 0.5, residual band 0.5: the
                 initial safe set of the warm-start / coarse-to-fine study.
  upd_d08_band   the update of that study to bound 0.8 started on the coarse
                 grid: c2f_d05_band's 61^4 value restricted to 21^4 (stored
                 here in full, FP64, as the warm start both sides take), warm
                 solve there, then -> 41^4 -> 61^4.
  mix5_31_band   problem 5 of the seeded 256-problem mix: 31^4, bound
                 0.7837..., residual band 0.5, cold.
  z2d_101_d05    the 2-D vertical quadcopter on 101^2, bound 0.5, cold,
                 stop over every node.
  z2d_chain_d05  51^2 cold -> 101^2, bound 0.5: the z-subsystem of the
                 decomposed near-hover quadcopter's initial safe set.
  z2d_mix0       the first 2-D problem of the seeded 256-problem mix, cold.

Per level the file holds the oracle's step count, dt, alpha and its last
eight residuals, the packed signs (V >= 0) of the FP64 value at every node,
and the value itself rounded to the nearest float32 (|rounding| <= 2.4e-7
for |V| <= 4), either at every node or, for the 41^4 and 61^4 levels of the
61^4 chains, at 2^18 nodes drawn with numpy default_rng(20210115) (their
flat indices are stored too).

Run from the repository root:  python tests/golden/make_goldens.py [case ...]
(about 40 minutes of single-threaded oracle time per 61^4 chain; the cases
run in parallel processes).
"""
from __future__ import annotations

import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2101_05916_amd import workloads as W  # noqa: E402

SAMPLE = 1 << 18
SAMPLE_SEED = 20210115


def sample_index(N: int) -> np.ndarray:
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(N, size=min(SAMPLE, N), replace=False)).astype(np.int64)


def _grid(P):
    return O.make_grid(P.n, P.lo, P.hi)


def chain(Ps, V0=None):
    """Coarse-to-fine oracle solve over the problems Ps (same box): level 0
    from V0 (None = cold), level k from the interpolated level k-1 value
    (the solve takes min(l, .) of its start)."""
    out = []
    start = V0
    for k, P in enumerate(Ps):
        if k > 0:
            start = O.interp(_grid(Ps[k - 1]), out[-1]["V"], _grid(P))
        t0 = time.perf_counter()
        r = O.solve(O.make_dyn(P.kind, P.params), _grid(P), P.l, P.dlo, P.dhi, tol=P.tol,
                    V0=start, band=P.band, history=True)
        r["seconds"] = time.perf_counter() - t0
        if r["status"] != O.OK:
            raise RuntimeError(f"oracle did not converge on {P.n}: status {r['status']}")
        print(f"  {P.name} {P.n[0]}^{len(P.n)}: {r['iterations']} steps, "
              f"{r['seconds']:.0f} s", flush=True)
        out.append(r)
    return out


def pack(levels, Ps, sampled, extra=None):
    d = {}
    d["levels"] = np.array([P.n[0] for P in Ps], dtype=np.int64)
    d["level_iterations"] = np.array([r["iterations"] for r in levels], dtype=np.int64)
    d["level_seconds"] = np.array([r["seconds"] for r in levels])
    d["dt"] = np.array([r["dt"] for r in levels])
    d["alpha"] = np.array([r["alpha"] for r in levels])
    d["res_tail"] = np.array([np.pad(r["res_hist"][-8:], (8 - min(8, len(r["res_hist"])), 0))
                              for r in levels])
    d["dbar"] = np.array([P.dhi[0] for P in Ps])
    d["band"] = np.array([P.band for P in Ps])
    for k, (r, P) in enumerate(zip(levels, Ps)):
        V = r["V"]
        d[f"sign{k}"] = np.packbits(V >= 0)
        if sampled[k]:
            idx = sample_index(V.size)
            d[f"idx{k}"] = idx
            d[f"V{k}"] = V[idx].astype(np.float32)
        else:
            d[f"V{k}"] = V.astype(np.float32)
    for k, v in (extra or {}).items():
        d[k] = v
    return d


def case_chain_d05():
    Ps = [W.quad_x4d(n, 0.5, "x") for n in (21, 41)]
    return pack(chain(Ps), Ps, [False, False])


def c2f_d05_problems():
    return [W.quad_x4d(n, 0.5, "x", band=W.BAND_4D_UPDATE) for n in (21, 41, 61)]


def upd_d08_problems():
    return [W.quad_x4d(n, 0.8, "x", band=W.BAND_4D_UPDATE) for n in (21, 41, 61)]


def case_c2f_and_update():
    Ps = c2f_d05_problems()
    lv = chain(Ps)
    first = pack(lv, Ps, [False, True, True])
    Qs = upd_d08_problems()
    warm = O.interp(_grid(Ps[-1]), lv[-1]["V"], _grid(Qs[0]))
    lq = chain(Qs, V0=warm)
    second = pack(lq, Qs, [False, True, True], extra={"warm21": warm})
    return first, second


def mix5_problem():
    e = W.batch_manifest(256, seed=0)[5]
    return W.problem_from_manifest(e)


def case_mix5():
    P = mix5_problem()
    return pack(chain([P]), [P], [False])


def case_z2d():
    P = W.quad_z2d(101, 0.5, "z")
    a = pack(chain([P]), [P], [False])
    Ps = [W.quad_z2d(n, 0.5, "z") for n in (51, 101)]
    b = pack(chain(Ps), Ps, [False, False])
    man = W.batch_manifest(256, seed=0)
    e = next(e for e in man if e["kind"] == W.QUAD_Z2D)
    Q = W.problem_from_manifest(e)
    c = pack(chain([Q]), [Q], [False], extra={"mix_index": np.array([e["index"]])})
    return a, b, c


def _run(name):
    t0 = time.perf_counter()
    print(f"{name}: start", flush=True)
    if name == "chain_d05":
        res = {"x4d_chain_d05": case_chain_d05()}
    elif name == "c2f":
        a, b = case_c2f_and_update()
        res = {"x4d_c2f_d05_band": a, "x4d_upd_d08_band": b}
    elif name == "mix5":
        res = {"x4d_mix5_31_band": case_mix5()}
    elif name == "z2d":
        a, b, c = case_z2d()
        res = {"z2d_101_d05": a, "z2d_chain_d05": b, "z2d_mix0": c}
    else:
        raise ValueError(name)
    for fname, d in res.items():
        np.savez_compressed(os.path.join(HERE, fname + ".npz"), **d)
    print(f"{name}: done in {time.perf_counter() - t0:.0f} s", flush=True)
    return name


if __name__ == "__main__":
    names = sys.argv[1:] or ["c2f", "chain_d05", "mix5", "z2d"]
    with Pool(len(names)) as pool:
        pool.map(_run, names)
