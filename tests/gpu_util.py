"""Helpers shared by the GPU parity tests: run a workload problem through the
device library and through the oracle on identical inputs."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2101_05916_amd import hjr


def ogrid(P):
    return O.make_grid(P.n, P.lo, P.hi)


def odyn(P):
    return O.make_dyn(P.kind, P.params)


def oracle_solve(P, V0=None, max_iter=100000, order=2, history=False, l=None):
    return O.solve(odyn(P), ogrid(P), P.l if l is None else l, P.dlo, P.dhi, tol=P.tol,
                   V0=V0, order=order, max_iter=max_iter, history=history, band=P.band)


def device_solve(P, dtype, V0=None, max_iter=100000, order=2, flags=0, chunk=0, l_host=None):
    import torch
    l_src = P.l if l_host is None else l_host
    l = torch.tensor(np.asarray(l_src, dtype=np.float64), dtype=dtype, device="cuda")
    v0 = None if V0 is None else torch.tensor(np.asarray(V0), dtype=dtype, device="cuda")
    V, st = hjr.solve(hjr.Spec.of(P), l, V0=v0, dtype=dtype, max_iter=max_iter, order=order,
                      flags=flags, chunk=chunk)
    torch.cuda.synchronize()
    return V.cpu().numpy().astype(np.float64), st


def zero_level_disagreement(Va, Vb):
    return float(np.mean((np.asarray(Va) >= 0) != (np.asarray(Vb) >= 0)))


def iterations_match(it_dev, ref):
    """Step counts must be equal; the one allowed exception is a device FP32
    run whose stopping residual sits within 1e-3 (relative) of tol in the
    oracle, where +-1 step is accepted."""
    if it_dev == ref["iterations"]:
        return True
    h = ref.get("res_hist")
    if h is None or abs(it_dev - ref["iterations"]) != 1:
        return False
    tol = 1e-4
    k = ref["iterations"] - 1
    near = [abs(h[i] - tol) <= 1e-3 * tol for i in (k - 1, k) if 0 <= i < len(h)]
    return any(near)
