"""Autotuner of the plane-tile height and the chunk length of the solver.

Two launch parameters of libhjr change speed but never results:

* ``tile_rows`` -- the stage kernels cut every plane of the two fastest grid
  axes into tiles of this many rows, each staged in LDS with two halo rows
  on either side (hjr_opts.tile_rows, hjr_problem.tile_rows).  Tall tiles
  stage fewer halo rows per node; short tiles make more tiles to spread over
  the compute units.
* ``chunk`` -- RK2 steps enqueued between two host reads of the residuals
  (hjr_opts.chunk).  Long chunks amortise launches and host round trips;
  the steps past a problem's stop step are skipped on the device, so their
  cost is a few empty launches.

``tune()`` measures candidates through the C ABI on the GPU at hand: the
device time of the stage launches (HJR_FLAG_PROFILE) for each tile height,
then the wall time per step for each chunk length with the chosen height,
and records the winners per (model, dtype, grid shape) in a JSON table.
The binding reads the table (``lookup``) when a call leaves tile_rows or
chunk unset; shapes missing from it take the nearest tuned shape of the same
model, dtype and dimension, or the library defaults.

    python -m paper_2101_05916_amd.autotune --out paper_2101_05916_amd/tuned.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
ROW_CANDIDATES = (1, 2, 3, 4, 6, 8, 10, 12, 14)
CHUNK_CANDIDATES = (4, 8, 16, 32, 64)

_cache = None


def key(kind: int, dtype_code: int, n) -> str:
    return f"{int(kind)}:{'f32' if dtype_code == 0 else 'f64'}:{'x'.join(str(int(x)) for x in n)}"


def load(path: str = TABLE) -> dict:
    global _cache
    if _cache is None or _cache[0] != path:
        try:
            with open(path) as fh:
                _cache = (path, json.load(fh).get("entries", {}))
        except (OSError, ValueError):
            _cache = (path, {})
    return _cache[1]


def lookup(kind: int, dtype_code: int, n, path: str = TABLE):
    """Tuned {"tile_rows", "chunk"} for this shape, else the entry of the
    nearest tuned node count with the same model, dtype and dimension, else
    None."""
    tab = load(path)
    k = key(kind, dtype_code, n)
    if k in tab:
        return tab[k]
    size = float(np.prod(n))
    best, bd = None, None
    for kk, v in tab.items():
        kd, dt, shape = kk.split(":")
        dims = [int(x) for x in shape.split("x")]
        if int(kd) != int(kind) or dt != k.split(":")[1] or len(dims) != len(n):
            continue
        d = abs(np.log(float(np.prod(dims)) / size))
        if bd is None or d < bd:
            best, bd = v, d
    return best


def row_candidates(n):
    nc = int(n[-1])
    return [r for r in ROW_CANDIDATES if r * nc <= 512 and (r + 4) * nc <= 1024] or [1]


def _stage_us(hjr, spec, l, rows, steps, dtype):
    flags = hjr.FLAG_PROFILE | hjr.FLAG_NO_PIPELINE
    hjr.solve(spec, l, dtype=dtype, max_iter=8, flags=flags, tile_rows=rows, chunk=8)
    _, st = hjr.solve(spec, l, dtype=dtype, max_iter=steps, flags=flags, tile_rows=rows, chunk=8)
    k, nl = st["kernel_ms"], st["kernel_launches"]
    return 1e3 * (k[0] / max(nl[0], 1) + k[1] / max(nl[1], 1))


def _wall_us(torch, hjr, spec, l, rows, chunk, steps, dtype):
    hjr.solve(spec, l, dtype=dtype, max_iter=chunk, tile_rows=rows, chunk=chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = hjr.solve(spec, l, dtype=dtype, max_iter=steps, tile_rows=rows, chunk=chunk)
    torch.cuda.synchronize()
    return 1e6 * (time.perf_counter() - t0) / max(st["iterations"], 1)


def choose_rows(stage_us):
    """Tile height with the least device time per step (ties: the taller)."""
    return min(stage_us, key=lambda r: (stage_us[r], -int(r)))


def choose_chunk(wall_us):
    """The shortest chunk within 2% of the least wall time per step: a solve
    overshoots its stop step by up to a chunk of (skipped) launches, so a
    shorter chunk wins when the per-step rates tie."""
    best = min(wall_us.values())
    return min(int(k) for k, v in wall_us.items() if v <= 1.02 * best)


def tune(problems, dtypes=("f32",), steps=64, log=print):
    """problems: workload Problem objects (model, grid, bounds).  The steps
    run from l with max_iter set, so the measured solves never converge."""
    import torch

    from . import hjr
    out = {}
    for P in problems:
        spec = hjr.Spec.of(P)
        for dts in dtypes:
            dtype = torch.float32 if dts == "f32" else torch.float64
            l = torch.tensor(P.l, dtype=dtype, device="cuda")
            rows = {r: _stage_us(hjr, spec, l, r, steps, dtype) for r in row_candidates(P.n)}
            best_r = choose_rows(rows)
            walls = {k: _wall_us(torch, hjr, spec, l, best_r, k, max(steps, 4 * k), dtype)
                     for k in CHUNK_CANDIDATES}
            best_k = choose_chunk(walls)
            e = {"tile_rows": int(best_r), "chunk": int(best_k),
                 "stage_us": {str(r): round(v, 2) for r, v in rows.items()},
                 "step_wall_us": {str(k): round(v, 2) for k, v in walls.items()}}
            out[key(P.kind, 0 if dts == "f32" else 1, P.n)] = e
            log(f"{P.name} {tuple(P.n)} {dts}: tile_rows {best_r} ({rows[best_r]:.1f} us/step), "
                f"chunk {best_k} ({walls[best_k]:.1f} us/step wall)")
    return out


def default_problems():
    """The grid classes of the workloads: 2-D 51^2..201^2 and 4-D 21^4..61^4,
    and the 10-D model's x-subsystem at 21^4..61^4."""
    from . import workloads as W
    return ([W.quad_z2d(n, 0.5, f"z{n}") for n in (51, 101, 151, 201)] +
            [W.quad_x4d(n, 0.5, f"x{n}") for n in (21, 31, 41, 51, 61)] +
            [W.quad_x4dv(n, 0.3, f"xv{n}") for n in (21, 41, 61)])


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--dtypes", default="f32")
    ap.add_argument("--steps", type=int, default=64)
    a = ap.parse_args()
    import torch
    dev = torch.cuda.get_device_properties(0)
    entries = tune(default_problems(), tuple(a.dtypes.split(",")), a.steps,
                   log=lambda s: print(s, flush=True))
    doc = {"device": dev.name, "gcn_arch": getattr(dev, "gcnArchName", ""),
           "note": "tile_rows: least device time of the two stage launches per step; "
                   "chunk: shortest within 2% of the least wall time per step",
           "entries": entries}
    with open(a.out, "w") as fh:
        json.dump(doc, fh, indent=1, sort_keys=True)
    print(f"wrote {a.out} ({len(entries)} entries)", flush=True)


if __name__ == "__main__":
    main()
