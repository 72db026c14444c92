"""hjr_solve_noalloc (the solve for callers that cannot allocate) against
hjr_solve_ex on the same inputs: bit-identical values, equal step counts,
residuals and statuses, over two calls in a row whose second problem is
smaller than the first (the scratch keeps the first call's contents), in
both precisions; plus the size limit and argument checks."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2101_05916_amd import hjr  # noqa: E402
from paper_2101_05916_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _solve_both(P, dtype, max_iter):
    spec = hjr.Spec.of(P)
    l = torch.tensor(P.l, dtype=dtype, device="cuda")
    V_ref, st_ref = hjr.solve(spec, l, dtype=dtype, max_iter=max_iter)
    V = torch.full_like(l, float("nan"))
    r, st = hjr.solve_noalloc(spec, l, V, max_iter=max_iter)
    torch.cuda.synchronize()
    return V_ref, st_ref, V, st, r


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_noalloc_matches_solve_two_calls(dtype):
    # first call: a 4-D problem stopped at max_iter; second: a smaller 2-D
    # problem solved to convergence
    cases = [(W.quad_x4d(21, 0.5), 60, hjr.NOT_CONVERGED), (W.quad_z2d(51, 0.5), 100000, hjr.OK)]
    for P, mi, want in cases:
        print(f"noalloc vs solve: {P.name} {P.n} {dtype} max_iter={mi}", flush=True)
        V_ref, st_ref, V, st, r = _solve_both(P, dtype, mi)
        assert r == want == st_ref["status"], (r, st_ref["status"])
        assert st["iterations"] == st_ref["iterations"]
        assert st["residual"] == st_ref["residual"]
        assert st["dt"] == st_ref["dt"]
        assert torch.equal(V, V_ref), float((V.double() - V_ref.double()).abs().max())


def test_noalloc_band_and_warm_start():
    # a warm start (V0) and the residual band go through the same path
    P = W.quad_x4d(21, 0.5, band=0.5)
    spec = hjr.Spec.of(P)
    l = torch.tensor(P.l, dtype=torch.float32, device="cuda")
    V0, _ = hjr.solve(spec, l, max_iter=50)
    spec8 = hjr.Spec.of(W.quad_x4d(21, 0.8, band=0.5))
    V_ref, st_ref = hjr.solve(spec8, l, V0=V0)
    V = torch.empty_like(l)
    r, st = hjr.solve_noalloc(spec8, l, V, V0=V0)
    torch.cuda.synchronize()
    assert r == hjr.OK == st_ref["status"]
    assert st["iterations"] == st_ref["iterations"]
    assert torch.equal(V, V_ref)


def test_noalloc_rejects_too_large_and_bad_input():
    # 61^4 in FP64 needs ~110 MB of stage-1 array: more than the scratch
    P = W.quad_x4d(61, 0.5)
    spec = hjr.Spec.of(P)
    assert P.size * 8 > hjr.NOALLOC_SCRATCH_BYTES
    l = torch.zeros(P.size, dtype=torch.float64, device="cuda")
    V = torch.zeros_like(l)
    r, _ = hjr.solve_noalloc(spec, l, V, check=False)
    assert r == hjr.ENOMEM
    assert torch.count_nonzero(V).item() == 0  # nothing was enqueued
    # invalid tolerance
    bad = hjr.Spec.of(W.quad_z2d(51, 0.5))
    bad.tol = -1.0
    l2 = torch.zeros(bad.size, dtype=torch.float32, device="cuda")
    r, _ = hjr.solve_noalloc(bad, l2, torch.zeros_like(l2), check=False)
    assert r == hjr.EINVAL
    L = hjr.lib()
    assert L.hjr_solve_noalloc(None, None, None, None, None, 1e-4, None, None, None) == hjr.EINVAL
