"""Host-side checks of the C ABI: the library loads without a GPU, exports
every entry point that include/hjr.h declares, the ctypes structs have the
C layouts, and argument validation rejects bad input before touching the
device."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_2101_05916_amd import hjr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hjr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hjr_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = hjr.lib()
    names = declared_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(hjr.EXPORTS)


def test_struct_layouts_match_c():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "hjr.h"
int main(void){
 printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(hjr_grid), sizeof(hjr_dyn),
   sizeof(hjr_dstb), sizeof(hjr_opts), sizeof(hjr_stats), sizeof(hjr_problem),
   sizeof(hjr_server_cfg), sizeof(hjr_request), sizeof(hjr_reply), sizeof(hjr_query),
   sizeof(hjr_subsystem), sizeof(hjr_query_decomposed));
 printf("%zu %zu %zu %zu %zu %zu %zu\n", offsetof(hjr_opts, flags),
   offsetof(hjr_stats, kernel_launches), offsetof(hjr_problem, tol), offsetof(hjr_request, cold),
   offsetof(hjr_problem, dfield), offsetof(hjr_request, dfield), offsetof(hjr_problem, order));
 return 0; }
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    got = [int(x) for x in out]
    want = [C.sizeof(hjr.Grid), C.sizeof(hjr.Dyn), C.sizeof(hjr.Dstb), C.sizeof(hjr.Opts),
            C.sizeof(hjr.Stats), C.sizeof(hjr.Problem), C.sizeof(hjr.ServerCfg),
            C.sizeof(hjr.Request), C.sizeof(hjr.Reply), C.sizeof(hjr.Query),
            C.sizeof(hjr.Subsystem), C.sizeof(hjr.QueryDecomposed),
            hjr.Opts.flags.offset, hjr.Stats.kernel_launches.offset, hjr.Problem.tol.offset,
            hjr.Request.cold.offset, hjr.Problem.dfield.offset, hjr.Request.dfield.offset,
            hjr.Problem.order.offset]
    assert got == want


def test_defaults_and_strerror():
    L = hjr.lib()
    o = hjr.Opts()
    assert L.hjr_opts_default(C.byref(o)) == hjr.OK
    assert (o.dtype, o.order, o.cfl, o.max_iter) == (hjr.F32, 2, 0.8, 100000)
    assert L.hjr_opts_default(None) == hjr.EINVAL
    for s in range(7):
        assert L.hjr_strerror(s)
    assert L.hjr_strerror(99) == b"unknown status"


def _opts(**kw):
    o = hjr.Opts()
    hjr.lib().hjr_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_workspace_bytes():
    L = hjr.lib()
    g = hjr.make_grid((41, 41, 41, 41), (-5, -2, -0.5, -2), (5, 2, 0.5, 2))
    out = C.c_size_t(0)
    assert L.hjr_workspace_bytes(C.byref(g), C.byref(_opts()), C.byref(out)) == hjr.OK
    assert out.value >= 41 ** 4 * 4
    out64 = C.c_size_t(0)
    assert L.hjr_workspace_bytes(C.byref(g), C.byref(_opts(dtype=hjr.F64)), C.byref(out64)) == hjr.OK
    assert out64.value > out.value
    bad = hjr.make_grid((2, 41), (0, 0), (1, 1))
    assert L.hjr_workspace_bytes(C.byref(bad), None, C.byref(out)) == hjr.EINVAL


@pytest.mark.parametrize("what", ["n<3", "lo>=hi", "ndim", "tol", "cfl", "order", "dstb",
                                  "kind", "null_l", "theta_range", "max_iter", "perm",
                                  "band<0", "band_nan"])
def test_solve_rejects_invalid_arguments_without_device(what):
    """Every one of these returns EINVAL before any HIP call (no GPU here)."""
    L = hjr.lib()
    n, lo, hi = [51, 51], [0.0, -4.0], [3.0, 4.0]
    kind, params = hjr.QUAD_Z2D, (0.91, 9.81, 7.0, 16.0)
    tol, kw = 1e-4, {}
    dlo, dhi = [-0.5], [0.5]
    lptr = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    if what == "n<3":
        n = [2, 51]
    elif what == "lo>=hi":
        hi = [0.0, 4.0]
    elif what == "ndim":
        n, lo, hi = [51] * 4, [0.0] * 4, [1.0] * 4
    elif what == "tol":
        tol = 0.0
    elif what == "cfl":
        kw = dict(cfl=1.5)
    elif what == "order":
        kw = dict(order=3)
    elif what == "dstb":
        dlo, dhi = [0.5], [-0.5]
    elif what == "kind":
        kind = 7
    elif what == "null_l":
        lptr = None
    elif what == "theta_range":
        kind, params = hjr.QUAD_X4D, (9.81, 8, 10, 10, 0.349)
        n, lo, hi = [11] * 4, [-5, -2, -2.0, -2], [5, 2, 2.0, 2]
    elif what == "max_iter":
        kw = dict(max_iter=0)
    elif what == "band<0":
        kw = dict(band=-0.5)
    elif what == "band_nan":
        kw = dict(band=float("nan"))
    elif what == "perm":
        kind = hjr.DI2X2
        params = (0.91, 9.81, 7, 16, 0.91, 9.81, 7, 16, 0, 1, 1, 3)
        n, lo, hi = [11] * 4, [0.0] * 4, [1.0] * 4
        dlo, dhi = [-0.5, -0.5], [0.5, 0.5]
    g = hjr.make_grid(n, lo, hi)
    dyn = hjr.make_dyn(kind, params)
    d = hjr.make_dstb(dlo, dhi)
    it = C.c_int64(0)
    res = C.c_double(0)
    r = L.hjr_solve(C.byref(dyn), C.byref(g), lptr, None, d, tol, C.byref(_opts(**kw)),
                    C.c_void_p(0x2000), C.byref(it), C.byref(res))
    assert r == hjr.EINVAL


@pytest.mark.parametrize("order", [-1, 3])
def test_batch_rejects_invalid_level_order_without_device(order):
    """A per-level derivative order outside 0..2 is EINVAL before any HIP call."""
    L = hjr.lib()
    p = hjr.Problem()
    p.dyn = hjr.make_dyn(hjr.QUAD_Z2D, (0.91, 9.81, 7.0, 16.0))
    p.nlev = 2
    for k in range(2):
        p.grids[k] = hjr.make_grid([51, 51], [0.0, -4.0], [3.0, 4.0])
        p.l[k] = 0x1000  # never dereferenced: validation fails first
        p.V[k] = 0x2000
    dd = hjr.make_dstb([-0.5], [0.5])
    p.d[0] = dd[0]
    p.tol = 1e-4
    p.order[1] = order
    assert L.hjr_solve_batch(1, C.byref(p), C.byref(_opts()), None) == hjr.EINVAL


def test_interp_and_mask_reject_invalid():
    L = hjr.lib()
    a = hjr.make_grid((11, 11), (0, 0), (1, 1))
    b = hjr.make_grid((21, 21), (0, 0), (1, 2))  # different box
    p = C.c_void_p(0x1000)
    q = C.c_void_p(0x2000)
    assert L.hjr_interp(C.byref(a), p, C.byref(b), q, None, None) == hjr.EINVAL
    assert L.hjr_interp(C.byref(a), p, C.byref(a), p, None, None) == hjr.EINVAL  # aliasing
    bad = hjr.make_grid((1, 11), (0, 0), (1, 1))
    assert L.hjr_refine_mask(C.byref(bad), p, q, None, None) == hjr.EINVAL


def test_field_solve_rejects_invalid_without_device():
    L = hjr.lib()
    dyn = hjr.make_dyn(hjr.QUAD_Z2D, (0.91, 9.81, 7.0, 16.0))
    g = (hjr.Grid * 1)(hjr.make_grid((11, 11), (0, -4), (3, 4)))
    p = (C.c_void_p * 1)(0x1000)
    q = (C.c_void_p * 1)(0x2000)
    none = (C.c_void_p * 1)(None)
    o = hjr.Opts()
    L.hjr_opts_default(C.byref(o))
    # missing field array, a missing level field, level counts out of range
    assert L.hjr_solve_field(C.byref(dyn), 1, g, p, None, None, 1e-4, C.byref(o), q, None) == hjr.EINVAL
    assert L.hjr_solve_field(C.byref(dyn), 1, g, p, none, None, 1e-4, C.byref(o), q, None) == hjr.EINVAL
    assert L.hjr_solve_field(C.byref(dyn), 0, g, p, p, None, 1e-4, C.byref(o), q, None) == hjr.EINVAL
    assert L.hjr_solve_field(C.byref(dyn), 5, g, p, p, None, 1e-4, C.byref(o), q, None) == hjr.EINVAL
    # the usual argument checks apply (tol, grid) before any device work
    assert L.hjr_solve_field(C.byref(dyn), 1, g, p, p, None, 0.0, C.byref(o), q, None) == hjr.EINVAL
    bad = (hjr.Grid * 1)(hjr.make_grid((2, 11), (0, -4), (3, 4)))
    assert L.hjr_solve_field(C.byref(dyn), 1, bad, p, p, None, 1e-4, C.byref(o), q, None) == hjr.EINVAL


def test_safety_query_rejects_invalid_without_device():
    L = hjr.lib()
    dyn = hjr.make_dyn(hjr.QUAD_Z2D, (0.91, 9.81, 7.0, 16.0))
    g = hjr.make_grid((11, 11), (0, -4), (3, 4))
    V = C.c_void_p(0x1000)
    o = hjr.Opts()
    L.hjr_opts_default(C.byref(o))
    q = hjr.Query()
    q.n = 0
    assert L.hjr_safety_query(C.byref(dyn), C.byref(g), V, C.byref(q), C.byref(o)) == hjr.OK
    q.n = -1
    assert L.hjr_safety_query(C.byref(dyn), C.byref(g), V, C.byref(q), C.byref(o)) == hjr.EINVAL
    q.n = 4  # states but no x
    assert L.hjr_safety_query(C.byref(dyn), C.byref(g), V, C.byref(q), C.byref(o)) == hjr.EINVAL
    q.x = 0x2000
    q.u_out = 0x3000  # filter output without a performance control
    assert L.hjr_safety_query(C.byref(dyn), C.byref(g), V, C.byref(q), C.byref(o)) == hjr.EINVAL
    q.u_out = None
    q.level = float("nan")
    assert L.hjr_safety_query(C.byref(dyn), C.byref(g), V, C.byref(q), C.byref(o)) == hjr.EINVAL
    q.level = 0.0
    o.order = 3
    assert L.hjr_safety_query(C.byref(dyn), C.byref(g), V, C.byref(q), C.byref(o)) == hjr.EINVAL
    o.order = 2
    bad = hjr.make_dyn(hjr.QUAD_X4D, (9.81, 8.0, 10.0, 10.0, 0.35))  # 4-D model on a 2-D grid
    assert L.hjr_safety_query(C.byref(bad), C.byref(g), V, C.byref(q), C.byref(o)) == hjr.EINVAL
    assert L.hjr_safety_query(C.byref(dyn), C.byref(g), None, C.byref(q), C.byref(o)) == hjr.EINVAL


def test_decomposed_query_rejects_invalid_without_device():
    L = hjr.lib()
    zx = hjr.make_dyn(hjr.QUAD_X4DV, (9.81, 8.0, 10.0, 10.0, 0.244))
    zz = hjr.make_dyn(hjr.QUAD_Z2D, (1.0, 9.81, 5.9, 13.7))
    subs = (hjr.Subsystem * 2)()
    subs[0].dyn = zx
    subs[0].grid = hjr.make_grid((5, 5, 5, 5), (-3, -4, -0.5, -4), (3, 4, 0.5, 4))
    subs[0].V = 0x1000
    for a in range(4):
        subs[0].state_index[a] = a
    subs[0].control_index = 0
    subs[1].dyn = zz
    subs[1].grid = hjr.make_grid((9, 9), (0, -4.5), (3.2, 4.5))
    subs[1].V = 0x2000
    subs[1].state_index[0], subs[1].state_index[1] = 4, 5
    subs[1].control_index = 1
    q = hjr.QueryDecomposed()
    q.n, q.state_dim, q.control_dim = 0, 6, 2
    o = hjr.Opts()
    L.hjr_opts_default(C.byref(o))
    assert L.hjr_safety_query_decomposed(2, subs, C.byref(q), C.byref(o)) == hjr.OK  # nothing to do
    q.n = 3
    q.x = 0x3000
    assert L.hjr_safety_query_decomposed(2, subs, C.byref(q), C.byref(o)) == hjr.EINVAL  # no sub_value
    q.sub_value = 0x4000
    q.state_dim = 5  # component 5 out of range
    assert L.hjr_safety_query_decomposed(2, subs, C.byref(q), C.byref(o)) == hjr.EINVAL
    q.state_dim = 6
    subs[1].state_index[0] = 3  # overlaps the first subsystem
    assert L.hjr_safety_query_decomposed(2, subs, C.byref(q), C.byref(o)) == hjr.EINVAL
    subs[1].state_index[0] = 4
    q.control_dim = 1  # second subsystem's control past the vector
    assert L.hjr_safety_query_decomposed(2, subs, C.byref(q), C.byref(o)) == hjr.EINVAL
    q.control_dim = 2
    assert L.hjr_safety_query_decomposed(0, subs, C.byref(q), C.byref(o)) == hjr.EINVAL


def test_local_update_rejects_invalid_without_device():
    L = hjr.lib()
    dyn = hjr.make_dyn(hjr.QUAD_Z2D, (0.91, 9.81, 7.0, 16.0))
    g = hjr.make_grid((11, 11), (0, -4), (3, 4))
    p = C.c_void_p(0x1000)
    d = hjr.make_dstb((-0.5,), (0.5,))
    o = hjr.Opts()
    L.hjr_opts_default(C.byref(o))
    assert L.hjr_band_mask(C.byref(g), p, -1, p, None, C.byref(o)) == hjr.EINVAL
    assert L.hjr_band_mask(C.byref(g), None, 2, p, None, C.byref(o)) == hjr.EINVAL
    bad = hjr.make_grid((2, 11), (0, -4), (3, 4))
    assert L.hjr_band_mask(C.byref(bad), p, 2, p, None, C.byref(o)) == hjr.EINVAL
    # no mask, no output, invalid tol: nothing is launched
    assert L.hjr_solve_local(C.byref(dyn), C.byref(g), p, None, d, None, None, 1e-4, C.byref(o),
                             p, None) == hjr.EINVAL
    assert L.hjr_solve_local(C.byref(dyn), C.byref(g), p, None, d, None, p, 1e-4, C.byref(o),
                             None, None) == hjr.EINVAL
    assert L.hjr_solve_local(C.byref(dyn), C.byref(g), p, None, d, None, p, -1.0, C.byref(o),
                             p, None) == hjr.EINVAL


def test_batch_and_server_reject_invalid():
    L = hjr.lib()
    out = C.c_size_t(0)
    assert L.hjr_batch_workspace_bytes(0, None, None, C.byref(out)) == hjr.EINVAL
    assert L.hjr_solve_batch(0, None, None, None) == hjr.EINVAL
    h = C.c_void_p()
    cfg = hjr.ServerCfg()
    cfg.dtype = 5
    assert L.hjr_server_create(C.byref(cfg), C.byref(h)) == hjr.EINVAL
    assert L.hjr_server_submit(None, None, None) == hjr.EINVAL
    assert L.hjr_server_poll(None, 1, None) == hjr.EINVAL
    assert L.hjr_server_destroy(None) == hjr.EINVAL


def test_batch_binding_takes_the_arrays_precision():
    """solve_batch runs the kernels of the problems' precision: a batch that
    mixes FP32 and FP64 arrays, or a dtype that differs from theirs, is
    refused before anything is launched."""
    torch = pytest.importorskip("torch")
    from paper_2101_05916_amd import workloads as W
    P = W.quad_z2d(11, 0.5)
    spec = hjr.Spec.of(P)

    def prob(dt):
        l = torch.tensor(P.l, dtype=dt)
        return hjr.make_problem(spec, l, torch.empty_like(l), tile_rows=[1])

    p32, p64 = prob(torch.float32), prob(torch.float64)
    assert p32._dtype == torch.float32 and p64._dtype == torch.float64
    with pytest.raises(ValueError, match="mix dtypes"):
        hjr.solve_batch([p32, p64], chunk=4)
    with pytest.raises(ValueError, match="differs"):
        hjr.solve_batch([p64], dtype=torch.float32, chunk=4)
    l = torch.tensor(P.l, dtype=torch.float32)
    with pytest.raises(ValueError, match="mix dtypes"):
        hjr.make_problem(spec, l, torch.empty(P.size, dtype=torch.float64), tile_rows=[1])
