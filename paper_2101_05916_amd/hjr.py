"""Thin ctypes binding of libhjr (include/hjr.h).

Argument marshalling only: every step of a solve runs in the HIP kernels of
``libhjr.so``.  PyTorch supplies device memory and the current stream.  The
library must be built in-tree (``__graft_entry__.build()``); importing this
module on a machine without it raises immediately -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhjr.so")

OK, EINVAL, ENOMEM, NOT_CONVERGED, EDEVICE, EBUSY, ENOTFOUND = range(7)
F32, F64 = 0, 1
QUAD_Z2D, QUAD_X4D, DI2X2, QUAD_X4DV = 0, 1, 2, 3
FLAG_NO_GRAPH, FLAG_NO_PIPELINE, FLAG_PROFILE, FLAG_FLAT_TILES = 1, 2, 4, 8

EXPORTS = (
    "hjr_opts_default", "hjr_strerror", "hjr_workspace_bytes", "hjr_solve", "hjr_solve_ex",
    "hjr_interp", "hjr_refine_mask", "hjr_solve_levels", "hjr_batch_workspace_bytes",
    "hjr_solve_batch", "hjr_server_create", "hjr_server_submit", "hjr_server_poll",
    "hjr_server_wait", "hjr_server_read_value", "hjr_server_memory", "hjr_server_destroy",
    "hjr_solve_field", "hjr_safety_query", "hjr_safety_query_decomposed", "hjr_band_mask",
    "hjr_solve_local", "hjr_solve_noalloc",
)


class HjrError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 4), ("lo", C.c_double * 4),
                ("hi", C.c_double * 4)]


class Dyn(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("p", C.c_double * 16)]


class Dstb(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("order", C.c_int32), ("cfl", C.c_double),
                ("max_iter", C.c_int64), ("stream", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("chunk", C.c_int32), ("flags", C.c_int32),
                ("tile_rows", C.c_int32), ("walk", C.c_int32), ("band", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("residual", C.c_double), ("dt", C.c_double),
                ("alpha", C.c_double * 4), ("status", C.c_int32), ("levels", C.c_int32),
                ("level_iterations", C.c_int64 * 4), ("cell_updates", C.c_int64),
                ("device_ms", C.c_double), ("kernel_ms", C.c_double * 2),
                ("kernel_launches", C.c_int64 * 2), ("kernel_cell_updates", C.c_int64)]

    def as_dict(self) -> dict:
        return dict(iterations=self.iterations, residual=self.residual, dt=self.dt,
                    alpha=list(self.alpha), status=self.status, levels=self.levels,
                    level_iterations=list(self.level_iterations),
                    cell_updates=self.cell_updates, device_ms=self.device_ms,
                    kernel_ms=list(self.kernel_ms), kernel_launches=list(self.kernel_launches),
                    kernel_cell_updates=self.kernel_cell_updates)


class Problem(C.Structure):
    _fields_ = [("dyn", Dyn), ("nlev", C.c_int32), ("reserved", C.c_int32),
                ("grids", Grid * 4), ("l", C.c_void_p * 4), ("V", C.c_void_p * 4),
                ("V0", C.c_void_p), ("d", Dstb * 2), ("tol", C.c_double),
                ("tile_rows", C.c_int32 * 4), ("band", C.c_double), ("dfield", C.c_void_p * 4),
                ("order", C.c_int32 * 4)]


class Query(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("value", C.c_void_p),
                ("grad", C.c_void_p), ("u_star", C.c_void_p), ("u_perf", C.c_void_p),
                ("u_out", C.c_void_p), ("level", C.c_double)]


class Subsystem(C.Structure):
    _fields_ = [("dyn", Dyn), ("grid", Grid), ("V", C.c_void_p), ("state_index", C.c_int32 * 4),
                ("control_index", C.c_int32), ("reserved", C.c_int32)]


class QueryDecomposed(C.Structure):
    _fields_ = [("n", C.c_int64), ("state_dim", C.c_int32), ("control_dim", C.c_int32),
                ("x", C.c_void_p), ("sub_value", C.c_void_p), ("value", C.c_void_p),
                ("active", C.c_void_p), ("grad", C.c_void_p), ("u_star", C.c_void_p),
                ("u_perf", C.c_void_p), ("u_out", C.c_void_p), ("level", C.c_double)]


class ServerCfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_active", C.c_int32),
                ("dtype", C.c_int32), ("order", C.c_int32), ("chunk", C.c_int32),
                ("cfl", C.c_double), ("max_iter", C.c_int64), ("device", C.c_int32),
                ("flags", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("instance_id", C.c_uint64), ("dyn", Dyn), ("grid", Grid), ("l", C.c_void_p),
                ("d", Dstb * 2), ("tol", C.c_double), ("cold", C.c_int32),
                ("reserved", C.c_int32), ("band", C.c_double), ("dfield", C.c_void_p)]


class Reply(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_int32), ("iterations", C.c_int64),
                ("residual", C.c_double), ("latency_ms", C.c_double), ("queue_ms", C.c_double),
                ("warm", C.c_int32), ("reserved2", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Load libhjr.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first "
                          "(there is no non-HIP fallback)")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    st = C.c_int
    L.hjr_opts_default.restype = st
    L.hjr_opts_default.argtypes = [P(Opts)]
    L.hjr_strerror.restype = C.c_char_p
    L.hjr_strerror.argtypes = [st]
    L.hjr_workspace_bytes.restype = st
    L.hjr_workspace_bytes.argtypes = [P(Grid), P(Opts), P(C.c_size_t)]
    L.hjr_solve.restype = st
    L.hjr_solve.argtypes = [P(Dyn), P(Grid), C.c_void_p, C.c_void_p, P(Dstb), C.c_double,
                            P(Opts), C.c_void_p, P(C.c_int64), P(C.c_double)]
    L.hjr_solve_ex.restype = st
    L.hjr_solve_ex.argtypes = [P(Dyn), P(Grid), C.c_void_p, C.c_void_p, P(Dstb), C.c_double,
                               P(Opts), C.c_void_p, P(Stats)]
    L.hjr_solve_noalloc.restype = st
    L.hjr_solve_noalloc.argtypes = [P(Dyn), P(Grid), C.c_void_p, C.c_void_p, P(Dstb),
                                    C.c_double, P(Opts), C.c_void_p, P(Stats)]
    L.hjr_interp.restype = st
    L.hjr_interp.argtypes = [P(Grid), C.c_void_p, P(Grid), C.c_void_p, C.c_void_p, P(Opts)]
    L.hjr_refine_mask.restype = st
    L.hjr_refine_mask.argtypes = [P(Grid), C.c_void_p, C.c_void_p, P(C.c_int64), P(Opts)]
    L.hjr_solve_levels.restype = st
    L.hjr_solve_levels.argtypes = [P(Dyn), C.c_int32, P(Grid), P(C.c_void_p), C.c_void_p,
                                   P(Dstb), C.c_double, P(Opts), P(C.c_void_p), P(C.c_void_p),
                                   P(C.c_int64), P(Stats)]
    L.hjr_solve_field.restype = st
    L.hjr_solve_field.argtypes = [P(Dyn), C.c_int32, P(Grid), P(C.c_void_p), P(C.c_void_p),
                                  C.c_void_p, C.c_double, P(Opts), P(C.c_void_p), P(Stats)]
    L.hjr_safety_query.restype = st
    L.hjr_safety_query.argtypes = [P(Dyn), P(Grid), C.c_void_p, P(Query), P(Opts)]
    L.hjr_band_mask.restype = st
    L.hjr_band_mask.argtypes = [P(Grid), C.c_void_p, C.c_int32, C.c_void_p, P(C.c_int64), P(Opts)]
    L.hjr_solve_local.restype = st
    L.hjr_solve_local.argtypes = [P(Dyn), P(Grid), C.c_void_p, C.c_void_p, P(Dstb), C.c_void_p,
                                  C.c_void_p, C.c_double, P(Opts), C.c_void_p, P(Stats)]
    L.hjr_safety_query_decomposed.restype = st
    L.hjr_safety_query_decomposed.argtypes = [C.c_int32, P(Subsystem), P(QueryDecomposed), P(Opts)]
    L.hjr_batch_workspace_bytes.restype = st
    L.hjr_batch_workspace_bytes.argtypes = [C.c_int32, P(Problem), P(Opts), P(C.c_size_t)]
    L.hjr_solve_batch.restype = st
    L.hjr_solve_batch.argtypes = [C.c_int32, P(Problem), P(Opts), P(Stats)]
    L.hjr_server_create.restype = st
    L.hjr_server_create.argtypes = [P(ServerCfg), P(C.c_void_p)]
    L.hjr_server_submit.restype = st
    L.hjr_server_submit.argtypes = [C.c_void_p, P(Request), P(C.c_uint64)]
    L.hjr_server_poll.restype = st
    L.hjr_server_poll.argtypes = [C.c_void_p, C.c_uint64, P(Reply)]
    L.hjr_server_wait.restype = st
    L.hjr_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_double, P(Reply)]
    L.hjr_server_read_value.restype = st
    L.hjr_server_read_value.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_size_t]
    L.hjr_server_memory.restype = st
    L.hjr_server_memory.argtypes = [C.c_void_p, P(C.c_size_t), P(C.c_size_t)]
    L.hjr_server_destroy.restype = st
    L.hjr_server_destroy.argtypes = [C.c_void_p]
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().hjr_strerror(status).decode()


# ---------------------------------------------------------------------------
# struct builders
# ---------------------------------------------------------------------------

def make_grid(n, lo, hi) -> Grid:
    g = Grid()
    g.ndim = len(n)
    for i in range(len(n)):
        g.n[i] = int(n[i])
        g.lo[i] = float(lo[i])
        g.hi[i] = float(hi[i])
    return g


def make_dyn(kind: int, params) -> Dyn:
    d = Dyn()
    d.kind = int(kind)
    for i, v in enumerate(params):
        d.p[i] = float(v)
    return d


def make_dstb(dlo, dhi):
    arr = (Dstb * 2)()
    dlo = np.atleast_1d(dlo)
    dhi = np.atleast_1d(dhi)
    for c in range(len(dlo)):
        arr[c].lo = float(dlo[c])
        arr[c].hi = float(dhi[c])
    return arr


def _torch():
    import torch
    return torch


def _dtype_code(dtype) -> int:
    torch = _torch()
    if dtype == torch.float32:
        return F32
    if dtype == torch.float64:
        return F64
    raise ValueError(f"unsupported dtype {dtype}")


def make_opts(dtype=None, order=2, cfl=0.8, max_iter=100000, chunk=0, flags=0, stream=None,
              tile_rows=0, band=0.0, walk=0) -> Opts:
    torch = _torch()
    o = Opts()
    lib().hjr_opts_default(C.byref(o))
    o.dtype = _dtype_code(dtype if dtype is not None else torch.float32)
    o.order = order
    o.cfl = cfl
    o.max_iter = max_iter
    o.chunk = chunk
    o.flags = flags
    o.tile_rows = tile_rows
    o.walk = walk
    o.band = band
    if stream is None:
        stream = torch.cuda.current_stream()
    o.stream = C.c_void_p(stream.cuda_stream)
    return o


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_tensor(t, n, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need contiguous {dtype} with {n} elements, got "
                         f"{t.dtype} {tuple(t.shape)}")


def channels(kind: int) -> int:
    """Disturbance channels of a model (1, or 2 for DI2X2)."""
    return 2 if kind == DI2X2 else 1


def _check_field(f, kind, n, dtype, name):
    """A per-node disturbance field: device tensor of 2 * channels * N
    elements (channel, lower/upper, node), contiguous, in the solve dtype."""
    _check_tensor(f.reshape(-1) if f.is_contiguous() else f, 2 * channels(kind) * n, dtype, name)


def _raise(status, what, allow=(OK,)):
    if status not in allow:
        raise HjrError(status, what)


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

@dataclass
class Spec:
    """Model + grid + bounds of one subsystem, in plain Python values."""
    kind: int
    params: tuple
    n: tuple
    lo: tuple
    hi: tuple
    dlo: tuple
    dhi: tuple
    tol: float = 1e-4
    band: float = 0.0   # residual band of the stop test, 0 = every node

    @classmethod
    def of(cls, p) -> "Spec":
        return cls(p.kind, tuple(p.params), tuple(p.n), tuple(p.lo), tuple(p.hi),
                   tuple(p.dlo), tuple(p.dhi), p.tol, float(getattr(p, "band", 0.0)))

    @property
    def size(self) -> int:
        return int(np.prod(self.n))


def workspace_bytes(spec: Spec, opts: Opts) -> int:
    out = C.c_size_t(0)
    g = make_grid(spec.n, spec.lo, spec.hi)
    _raise(lib().hjr_workspace_bytes(C.byref(g), C.byref(opts), C.byref(out)),
           "hjr_workspace_bytes")
    return out.value


def tuned(kind, dtype, n):
    """Autotuned {"tile_rows", "chunk"} for a grid shape (autotune.py), or {}."""
    from . import autotune
    return autotune.lookup(kind, _dtype_code(dtype), n) or {}


def solve(spec: Spec, l, V0=None, V_out=None, *, dtype=None, order=2, cfl=0.8,
          max_iter=100000, chunk=None, flags=0, workspace=True, check=True, tile_rows=None,
          dfield=None, walk=0):
    """One safe-set solve.  l, V0, V_out: device tensors of spec.size elements.
    dfield: optional per-node disturbance boxes, a device tensor of
    (channels, 2, spec.size) elements (hjr_solve_field); without it the
    constant boxes spec.dlo, spec.dhi apply.  chunk / tile_rows None take
    the autotuned values for this shape (library defaults if it was not
    tuned).  Returns (V_out, stats dict).  Raises HjrError on failure; a
    solve that hits max_iter returns with stats['status'] == NOT_CONVERGED."""
    torch = _torch()
    dtype = dtype or l.dtype
    if chunk is None or tile_rows is None:
        t = tuned(spec.kind, dtype, spec.n)
        chunk = t.get("chunk", 0) if chunk is None else chunk
        tile_rows = t.get("tile_rows", 0) if tile_rows is None else tile_rows
    N = spec.size
    _check_tensor(l, N, dtype, "l")
    if V0 is not None:
        _check_tensor(V0, N, dtype, "V0")
    if V_out is None:
        V_out = torch.empty(N, dtype=dtype, device=l.device)
    _check_tensor(V_out, N, dtype, "V_out")
    o = make_opts(dtype, order, cfl, max_iter, chunk, flags, tile_rows=tile_rows, band=spec.band,
                  walk=walk)
    ws = None
    if workspace:
        nb = workspace_bytes(spec, o)
        ws = torch.empty(nb, dtype=torch.uint8, device=l.device)
        o.workspace = C.c_void_p(ws.data_ptr())
        o.workspace_bytes = nb
    st = Stats()
    g = make_grid(spec.n, spec.lo, spec.hi)
    dyn = make_dyn(spec.kind, spec.params)
    if dfield is not None:
        _check_field(dfield, spec.kind, N, dtype, "dfield")
        lp = (C.c_void_p * 1)(l.data_ptr())
        fp = (C.c_void_p * 1)(dfield.data_ptr())
        vp = (C.c_void_p * 1)(V_out.data_ptr())
        r = lib().hjr_solve_field(C.byref(dyn), 1, C.byref(g), lp, fp, _ptr(V0), spec.tol,
                                  C.byref(o), vp, C.byref(st))
        what = "hjr_solve_field"
    else:
        d = make_dstb(spec.dlo, spec.dhi)
        r = lib().hjr_solve_ex(C.byref(dyn), C.byref(g), _ptr(l), _ptr(V0), d, spec.tol,
                               C.byref(o), _ptr(V_out), C.byref(st))
        what = "hjr_solve_ex"
    if check:
        _raise(r, what, (OK, NOT_CONVERGED))
    del ws
    out = st.as_dict()
    out["return"] = r
    return V_out, out


NOALLOC_SCRATCH_BYTES = 64 << 20  # HJR_NOALLOC_SCRATCH_BYTES


def solve_noalloc(spec: Spec, l, V_out, V0=None, *, order=2, cfl=0.8, max_iter=100000,
                  chunk=None, tile_rows=None, flags=0, check=True):
    """hjr_solve_noalloc: the solve of `solve` (constant bounds, one level)
    without any allocation in the library; l, V_out (and V0) are the
    caller's device tensors of spec.size elements, all of one dtype.  Runs
    on torch's current stream.  Returns (status, stats dict); raises
    HjrError unless the status is OK or NOT_CONVERGED (check=False returns
    any status)."""
    torch = _torch()
    dtype = l.dtype
    if chunk is None or tile_rows is None:
        t = tuned(spec.kind, dtype, spec.n)
        chunk = t.get("chunk", 0) if chunk is None else chunk
        tile_rows = t.get("tile_rows", 0) if tile_rows is None else tile_rows
    N = spec.size
    _check_tensor(l, N, dtype, "l")
    _check_tensor(V_out, N, dtype, "V_out")
    if V0 is not None:
        _check_tensor(V0, N, dtype, "V0")
    o = make_opts(dtype, order, cfl, max_iter, chunk, flags, tile_rows=tile_rows, band=spec.band,
                  stream=torch.cuda.current_stream(l.device))
    st = Stats()
    g = make_grid(spec.n, spec.lo, spec.hi)
    dyn = make_dyn(spec.kind, spec.params)
    d = make_dstb(spec.dlo, spec.dhi)
    r = lib().hjr_solve_noalloc(C.byref(dyn), C.byref(g), _ptr(l), _ptr(V0), d, spec.tol,
                                C.byref(o), _ptr(V_out), C.byref(st))
    if check:
        _raise(r, "hjr_solve_noalloc", (OK, NOT_CONVERGED))
    return r, st.as_dict()


def band_mask(spec: Spec, V, k: int):
    """Band of the previous value V (hjr_band_mask): a device uint8 tensor of
    spec.size nodes and the number of nodes in it."""
    torch = _torch()
    _check_tensor(V, spec.size, V.dtype, "V")
    m = torch.empty(spec.size, dtype=torch.uint8, device=V.device)
    cnt = C.c_int64(0)
    o = make_opts(V.dtype)
    g = make_grid(spec.n, spec.lo, spec.hi)
    _raise(lib().hjr_band_mask(C.byref(g), _ptr(V), int(k), _ptr(m), C.byref(cnt), C.byref(o)),
           "hjr_band_mask")
    return m, cnt.value


def solve_local(spec: Spec, l, mask, V0=None, V_out=None, *, dtype=None, order=2, cfl=0.8,
                max_iter=100000, chunk=None, flags=0, dfield=None):
    """Localized update (hjr_solve_local): only the nodes set in mask (device
    uint8, spec.size) are updated.  Returns (V_out, stats dict)."""
    torch = _torch()
    dtype = dtype or l.dtype
    N = spec.size
    _check_tensor(l, N, dtype, "l")
    _check_tensor(mask, N, torch.uint8, "mask")
    if V0 is not None:
        _check_tensor(V0, N, dtype, "V0")
    if V_out is None:
        V_out = torch.empty(N, dtype=dtype, device=l.device)
    if chunk is None:
        chunk = tuned(spec.kind, dtype, spec.n).get("chunk", 0)
    o = make_opts(dtype, order, cfl, max_iter, chunk, flags, band=spec.band)
    g = make_grid(spec.n, spec.lo, spec.hi)
    dyn = make_dyn(spec.kind, spec.params)
    d = make_dstb(spec.dlo, spec.dhi)
    if dfield is not None:
        _check_field(dfield, spec.kind, N, dtype, "dfield")
    st = Stats()
    r = lib().hjr_solve_local(C.byref(dyn), C.byref(g), _ptr(l), _ptr(V0), d, _ptr(dfield),
                              _ptr(mask), spec.tol, C.byref(o), _ptr(V_out), C.byref(st))
    _raise(r, "hjr_solve_local", (OK, NOT_CONVERGED))
    out = st.as_dict()
    out["return"] = r
    return V_out, out


def solve_levels(spec: Spec, grids_n, ls, V0=None, *, dtype=None, order=2, cfl=0.8,
                 max_iter=100000, chunk=0, flags=0, masks=False, dfields=None, walk=0):
    """Coarse-to-fine solve: grids_n is a list of per-level node counts over
    spec's box, ls the per-level constraints, dfields optional per-level
    disturbance fields (hjr_solve_field; no masks then).  Returns (list of V
    per level, list of masks or None, mask counts, stats)."""
    torch = _torch()
    nlev = len(grids_n)
    dtype = dtype or ls[0].dtype
    grids = (Grid * nlev)(*[make_grid(n, spec.lo, spec.hi) for n in grids_n])
    Vs = [torch.empty(int(np.prod(n)), dtype=dtype, device=ls[0].device) for n in grids_n]
    for k in range(nlev):
        _check_tensor(ls[k], int(np.prod(grids_n[k])), dtype, f"l[{k}]")
    lp = (C.c_void_p * nlev)(*[t.data_ptr() for t in ls])
    vp = (C.c_void_p * nlev)(*[t.data_ptr() for t in Vs])
    mk = None
    mp = None
    counts = (C.c_int64 * nlev)()
    if masks:
        mk = [torch.zeros(int(np.prod([x - 1 for x in n])), dtype=torch.uint8,
                          device=ls[0].device) for n in grids_n]
        mp = (C.c_void_p * nlev)(*[t.data_ptr() for t in mk])
    o = make_opts(dtype, order, cfl, max_iter, chunk, flags, band=spec.band, walk=walk)
    st = Stats()
    dyn = make_dyn(spec.kind, spec.params)
    if dfields is not None:
        if masks:
            raise ValueError("hjr_solve_field produces no refinement masks")
        for k in range(nlev):
            _check_field(dfields[k], spec.kind, int(np.prod(grids_n[k])), dtype, f"dfields[{k}]")
        fp = (C.c_void_p * nlev)(*[t.data_ptr() for t in dfields])
        r = lib().hjr_solve_field(C.byref(dyn), nlev, grids, lp, fp, _ptr(V0), spec.tol,
                                  C.byref(o), vp, C.byref(st))
        _raise(r, "hjr_solve_field", (OK, NOT_CONVERGED))
    else:
        d = make_dstb(spec.dlo, spec.dhi)
        r = lib().hjr_solve_levels(C.byref(dyn), nlev, grids, lp, _ptr(V0), d, spec.tol,
                                   C.byref(o), vp, mp, counts if masks else None, C.byref(st))
        _raise(r, "hjr_solve_levels", (OK, NOT_CONVERGED))
    out = st.as_dict()
    out["return"] = r
    return Vs, mk, (list(counts) if masks else None), out


def make_problem(spec: Spec, l, V_out, V0=None, levels=None, tile_rows=None,
                 dtype=None, dfields=None, orders=None) -> Problem:
    """levels: optional list of (n, l_k, V_k) for a coarse-to-fine job; else
    one level with (spec.n, l, V_out).  tile_rows None takes the autotuned
    height of every level's shape (dtype: that of the level arrays).
    dfields: optional per-level disturbance fields (entries may be None).
    orders: optional per-level derivative order (1, 2, or 0 = the batch's)."""
    p = Problem()
    p.dyn = make_dyn(spec.kind, spec.params)
    if levels is None:
        levels = [(spec.n, l, V_out)]
    dts = {t.dtype for _, lk, Vk in levels for t in (lk, Vk)}
    if len(dts) != 1:
        raise ValueError(f"make_problem: the level arrays mix dtypes {sorted(map(str, dts))}")
    p._dtype = dts.pop()  # solve_batch runs the kernels of this precision
    p.nlev = len(levels)
    for k, (n, lk, Vk) in enumerate(levels):
        p.grids[k] = make_grid(n, spec.lo, spec.hi)
        p.l[k] = lk.data_ptr()
        p.V[k] = Vk.data_ptr()
    p.V0 = V0.data_ptr() if V0 is not None else None
    dd = make_dstb(spec.dlo, spec.dhi)
    p.d[0] = dd[0]
    p.d[1] = dd[1]
    p.tol = spec.tol
    p.band = spec.band
    if tile_rows is None:
        tile_rows = [tuned(spec.kind, dtype or lk.dtype, n).get("tile_rows", 0)
                     for n, lk, _ in levels]
    for k, r in enumerate(tile_rows):
        p.tile_rows[k] = int(r)
    for k, f in enumerate(dfields or []):
        if f is not None:
            n, lk, _ = levels[k]
            _check_field(f, spec.kind, int(np.prod(n)), lk.dtype, f"dfields[{k}]")
            p.dfield[k] = f.data_ptr()
    for k, o in enumerate(orders or []):
        p.order[k] = int(o)
    return p


def solve_batch(problems, *, dtype=None, order=2, cfl=0.8, max_iter=100000, chunk=None,
                flags=0, device=None, walk=0):
    """problems: list of Problem structs (make_problem).  dtype None takes the
    precision of the problems' arrays (all alike); a dtype that differs from
    it is an error.  chunk None takes the autotuned chunk of the largest grid
    in the batch.  Returns (return status, list of stats dicts)."""
    torch = _torch()
    have = {getattr(p, "_dtype", None) for p in problems} - {None}
    if len(have) > 1:
        raise ValueError(f"solve_batch: the problems mix dtypes {sorted(map(str, have))}")
    if dtype is None:
        dtype = have.pop() if have else torch.float32
    elif have and dtype not in have:
        raise ValueError(f"solve_batch: dtype {dtype} differs from the problems' arrays ({have.pop()})")
    n = len(problems)
    if chunk is None:
        big = max(problems, key=lambda p: max(int(np.prod([p.grids[k].n[i] for i in range(p.grids[k].ndim)]))
                                             for k in range(p.nlev)))
        g = big.grids[big.nlev - 1]
        chunk = tuned(big.dyn.kind, dtype or torch.float32,
                      [g.n[i] for i in range(g.ndim)]).get("chunk", 0)
    arr = (Problem * n)(*problems)
    o = make_opts(dtype or torch.float32, order, cfl, max_iter, chunk, flags, walk=walk)
    nb = C.c_size_t(0)
    _raise(lib().hjr_batch_workspace_bytes(n, arr, C.byref(o), C.byref(nb)),
           "hjr_batch_workspace_bytes")
    ws = torch.empty(nb.value, dtype=torch.uint8, device=device or "cuda")
    o.workspace = C.c_void_p(ws.data_ptr())
    o.workspace_bytes = nb.value
    res = (Stats * n)()
    r = lib().hjr_solve_batch(n, arr, C.byref(o), res)
    _raise(r, "hjr_solve_batch", (OK, NOT_CONVERGED))
    del ws
    return r, [res[i].as_dict() for i in range(n)]


def interp(src_n, Vs, dst_n, lo, hi, l_dst=None, out=None):
    torch = _torch()
    src = make_grid(src_n, lo, hi)
    dst = make_grid(dst_n, lo, hi)
    Nd = int(np.prod(dst_n))
    if out is None:
        out = torch.empty(Nd, dtype=Vs.dtype, device=Vs.device)
    o = make_opts(Vs.dtype)
    _raise(lib().hjr_interp(C.byref(src), _ptr(Vs), C.byref(dst), _ptr(out), _ptr(l_dst),
                            C.byref(o)), "hjr_interp")
    return out


def refine_mask(n, lo, hi, V):
    torch = _torch()
    g = make_grid(n, lo, hi)
    m = torch.empty(int(np.prod([x - 1 for x in n])), dtype=torch.uint8, device=V.device)
    cnt = C.c_int64(0)
    o = make_opts(V.dtype)
    _raise(lib().hjr_refine_mask(C.byref(g), _ptr(V), _ptr(m), C.byref(cnt), C.byref(o)),
           "hjr_refine_mask")
    return m, cnt.value


# ---------------------------------------------------------------------------
# safety queries
# ---------------------------------------------------------------------------

def controls(kind: int) -> int:
    """Control inputs of a model (1, or 2 for DI2X2)."""
    return 2 if kind == DI2X2 else 1


def query(spec: Spec, V, X, *, order=2, u_perf=None, level=0.0, grad=True, u_star=True,
          stream=None, out=None):
    """Safety query (hjr_safety_query) at the states X (device float64
    tensor, n x ndim) on the converged value V (device tensor of spec.size
    elements, float32 or float64).  Returns a dict of device float64 tensors:
    value (n,), grad (n, ndim), u_star (n, controls) and, when u_perf
    (n, controls) is given, u_out = u_perf where value >= level else u_star.
    out: optional dict of preallocated output tensors of those names.
    Asynchronous on the stream (default: the current one)."""
    torch = _torch()
    _check_tensor(V, spec.size, V.dtype, "V")
    D = len(spec.n)
    m = controls(spec.kind)
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float64
            and X.is_contiguous() and X.dim() == 2 and X.shape[1] == D):
        raise ValueError(f"X must be a contiguous CUDA float64 tensor of shape (n, {D})")
    n = X.shape[0]
    res = dict(out or {})
    dev = X.device

    def buf(name, shape, want):
        if not want:
            return None
        if name not in res:
            res[name] = torch.empty(shape, dtype=torch.float64, device=dev)
        return res[name]

    q = Query()
    q.n = n
    q.x = X.data_ptr()
    q.value = buf("value", (n,), True).data_ptr()
    g = buf("grad", (n, D), grad)
    q.grad = g.data_ptr() if g is not None else None
    u = buf("u_star", (n, m), u_star)
    q.u_star = u.data_ptr() if u is not None else None
    if u_perf is not None:
        if not (u_perf.is_cuda and u_perf.dtype == torch.float64 and u_perf.is_contiguous()
                and u_perf.numel() == n * m):
            raise ValueError(f"u_perf must be a contiguous CUDA float64 tensor of {n} x {m}")
        q.u_perf = u_perf.data_ptr()
        q.u_out = buf("u_out", (n, m), True).data_ptr()
    q.level = float(level)
    o = make_opts(V.dtype, order, stream=stream)
    g_ = make_grid(spec.n, spec.lo, spec.hi)
    dyn = make_dyn(spec.kind, spec.params)
    _raise(lib().hjr_safety_query(C.byref(dyn), C.byref(g_), _ptr(V), C.byref(q), C.byref(o)),
           "hjr_safety_query")
    return res


def query_decomposed(subsystems, X, *, control_dim=None, order=2, u_perf=None, level=0.0,
                     stream=None, out=None):
    """Decomposed safety query (hjr_safety_query_decomposed).  subsystems:
    list of (spec, V, state_index, control_index); X: device float64 tensor
    (n, state_dim).  Returns a dict of device tensors: sub_value (n, nsub),
    value (n,), active (n,) int32, grad (n, state_dim), u_star (n,
    control_dim) and, with u_perf, u_out."""
    torch = _torch()
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float64
            and X.is_contiguous() and X.dim() == 2):
        raise ValueError("X must be a contiguous CUDA float64 tensor (n, state_dim)")
    n, dim = X.shape
    ns = len(subsystems)
    if control_dim is None:
        control_dim = max(c + controls(sp.kind) for sp, _, _, c in subsystems)
    arr = (Subsystem * ns)()
    vdtype = None
    for k, (sp, V, idx, c) in enumerate(subsystems):
        _check_tensor(V, sp.size, V.dtype, f"V[{k}]")
        if vdtype is not None and V.dtype != vdtype:
            raise ValueError("every subsystem value must have the same dtype")
        vdtype = V.dtype
        arr[k].dyn = make_dyn(sp.kind, sp.params)
        arr[k].grid = make_grid(sp.n, sp.lo, sp.hi)
        arr[k].V = V.data_ptr()
        for a, ci in enumerate(idx):
            arr[k].state_index[a] = int(ci)
        arr[k].control_index = int(c)
    res = dict(out or {})
    dev = X.device

    def buf(name, shape, dt=torch.float64):
        if name not in res:
            res[name] = torch.empty(shape, dtype=dt, device=dev)
        return res[name].data_ptr()

    q = QueryDecomposed()
    q.n = n
    q.state_dim = dim
    q.control_dim = control_dim
    q.x = X.data_ptr()
    q.sub_value = buf("sub_value", (n, ns))
    q.value = buf("value", (n,))
    q.active = buf("active", (n,), torch.int32)
    q.grad = buf("grad", (n, dim))
    q.u_star = buf("u_star", (n, control_dim))
    if u_perf is not None:
        if not (u_perf.is_cuda and u_perf.dtype == torch.float64 and u_perf.is_contiguous()
                and u_perf.numel() == n * control_dim):
            raise ValueError("u_perf must be a contiguous CUDA float64 tensor (n, control_dim)")
        q.u_perf = u_perf.data_ptr()
        q.u_out = buf("u_out", (n, control_dim))
    q.level = float(level)
    o = make_opts(vdtype, order, stream=stream)
    _raise(lib().hjr_safety_query_decomposed(ns, arr, C.byref(q), C.byref(o)),
           "hjr_safety_query_decomposed")
    return res


# ---------------------------------------------------------------------------
# server
# ---------------------------------------------------------------------------

class Server:
    """Continuous-batching safe-set update server (hjr_server_*)."""

    def __init__(self, hbm_budget_bytes=0, max_active=256, dtype=F32, order=2, chunk=0,
                 cfl=0.8, max_iter=100000, device=0, flags=0):
        c = ServerCfg()
        c.hbm_budget_bytes = hbm_budget_bytes
        c.max_active = max_active
        c.dtype = dtype
        c.order = order
        c.chunk = chunk
        c.cfl = cfl
        c.max_iter = max_iter
        c.device = device
        c.flags = flags
        self.dtype = dtype
        h = C.c_void_p()
        _raise(lib().hjr_server_create(C.byref(c), C.byref(h)), "hjr_server_create")
        self._h = h

    def submit(self, instance_id: int, spec: Spec, l_host=None, cold=False,
               dfield_host=None) -> int:
        """dfield_host: optional per-node disturbance boxes of this request,
        a host array of (channels, 2, N) values (copied before returning)."""
        req = Request()
        req.instance_id = instance_id
        req.dyn = make_dyn(spec.kind, spec.params)
        req.grid = make_grid(spec.n, spec.lo, spec.hi)
        keep = None
        if l_host is not None:
            keep = np.ascontiguousarray(l_host, dtype=np.float64 if self.dtype == F64 else np.float32)
            req.l = keep.ctypes.data
        fkeep = None
        if dfield_host is not None:
            fkeep = np.ascontiguousarray(dfield_host,
                                         dtype=np.float64 if self.dtype == F64 else np.float32)
            if fkeep.size != 2 * channels(spec.kind) * spec.size:
                raise ValueError("dfield_host must hold (channels, 2, N) values")
            req.dfield = fkeep.ctypes.data
        dd = make_dstb(spec.dlo, spec.dhi)
        req.d[0] = dd[0]
        req.d[1] = dd[1]
        req.tol = spec.tol
        req.band = spec.band
        req.cold = 1 if cold else 0
        t = C.c_uint64(0)
        _raise(lib().hjr_server_submit(self._h, C.byref(req), C.byref(t)), "hjr_server_submit")
        return t.value

    def poll(self, ticket: int):
        rep = Reply()
        r = lib().hjr_server_poll(self._h, ticket, C.byref(rep))
        if r == EBUSY:
            return None
        _raise(r, "hjr_server_poll")
        return _reply_dict(rep)

    def wait(self, ticket: int, timeout_ms: float = -1.0):
        rep = Reply()
        r = lib().hjr_server_wait(self._h, ticket, timeout_ms, C.byref(rep))
        if r == EBUSY:
            return None
        _raise(r, "hjr_server_wait")
        return _reply_dict(rep)

    def read_value(self, instance_id: int, size: int):
        out = np.empty(size, dtype=np.float64 if self.dtype == F64 else np.float32)
        _raise(lib().hjr_server_read_value(self._h, instance_id, out.ctypes.data, out.nbytes),
               "hjr_server_read_value")
        return out

    def memory(self):
        u = C.c_size_t(0)
        b = C.c_size_t(0)
        _raise(lib().hjr_server_memory(self._h, C.byref(u), C.byref(b)), "hjr_server_memory")
        return u.value, b.value

    def close(self):
        if self._h:
            r = lib().hjr_server_destroy(self._h)
            self._h = None
            _raise(r, "hjr_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _reply_dict(rep: Reply) -> dict:
    return dict(status=rep.status, iterations=rep.iterations, residual=rep.residual,
                latency_ms=rep.latency_ms, queue_ms=rep.queue_ms, warm=bool(rep.warm))
