"""ctypes wrapper of the FP64 CPU oracle (``hjr_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The product package
never imports it, and it imports nothing from the product package: the two
sides meet only through the seeded input generators, which hold none of the
method's arithmetic.

Every function mirrors one entry of ``hjr_oracle.h``; inputs are numpy
arrays (converted to contiguous float64), outputs are numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_SRC = os.path.join(_HERE, "hjr_oracle.c")

QUAD_Z2D, QUAD_X4D, DI2X2, QUAD_X4DV = 0, 1, 2, 3
OK, EINVAL, NOT_CONVERGED = 0, 1, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
            "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 4),
                ("lo", C.c_double * 4), ("hi", C.c_double * 4)]


class Dyn(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("p", C.c_double * 16)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        gp, yp = C.POINTER(Grid), C.POINTER(Dyn)
        L.orc_hamiltonian.restype = C.c_double
        L.orc_hamiltonian.argtypes = [yp, dp, dp, dp, dp]
        L.orc_dynamics.restype = None
        L.orc_dynamics.argtypes = [yp, dp, dp, dp, dp]
        L.orc_lf_alpha.restype = None
        L.orc_lf_alpha.argtypes = [yp, gp, dp, dp, dp]
        L.orc_dt.restype = C.c_double
        L.orc_dt.argtypes = [gp, dp, C.c_double]
        L.orc_line_derivs.restype = None
        L.orc_line_derivs.argtypes = [dp, C.c_int, C.c_double, C.c_int, dp, dp]
        L.orc_spatial_op.restype = None
        L.orc_spatial_op.argtypes = [yp, gp, dp, dp, dp, C.c_int, dp, dp]
        L.orc_iterate.restype = C.c_double
        L.orc_iterate.argtypes = [yp, gp, dp, dp, dp, C.c_double, C.c_int, dp, dp, dp]
        L.orc_iterate_at.restype = C.c_double
        L.orc_iterate_at.argtypes = [yp, gp, dp, dp, dp, C.c_double, C.c_int, dp, dp,
                                     C.c_int64]
        L.orc_solve.restype = C.c_int
        L.orc_solve.argtypes = [yp, gp, dp, dp, dp, dp, C.c_double, C.c_double, C.c_double,
                                C.c_int, C.c_int64, dp, C.POINTER(C.c_int64), dp, dp, dp,
                                dp, dp]
        L.orc_residual_band.restype = C.c_double
        L.orc_residual_band.argtypes = [C.c_int64, dp, dp, C.c_double]
        L.orc_interp.restype = C.c_int
        L.orc_interp.argtypes = [gp, dp, gp, dp]
        L.orc_refine_mask.restype = C.c_int64
        L.orc_refine_mask.argtypes = [gp, dp, C.POINTER(C.c_uint8)]
        L.orc_lf_alpha_field.restype = None
        L.orc_lf_alpha_field.argtypes = [yp, gp, dp, dp, dp, dp]
        L.orc_spatial_op_field.restype = None
        L.orc_spatial_op_field.argtypes = [yp, gp, dp, dp, dp, dp, C.c_int, dp, dp]
        L.orc_iterate_field.restype = C.c_double
        L.orc_iterate_field.argtypes = [yp, gp, dp, dp, dp, dp, C.c_double, C.c_int, dp, dp,
                                        dp]
        L.orc_iterate_at_field.restype = C.c_double
        L.orc_iterate_at_field.argtypes = [yp, gp, dp, dp, dp, dp, C.c_double, C.c_int, dp,
                                           dp, C.c_int64]
        L.orc_query_decomposed.restype = C.c_int
        L.orc_query_decomposed.argtypes = [C.c_int, yp, gp, C.POINTER(dp), C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int32), C.POINTER(dp), C.POINTER(dp),
                                           C.c_int, dp, C.c_double, dp, dp,
                                           C.POINTER(C.c_int32), dp, dp, dp, dp]
        L.orc_band_mask.restype = C.c_int64
        L.orc_band_mask.argtypes = [gp, dp, C.c_int, C.POINTER(C.c_uint8)]
        L.orc_solve_masked.restype = C.c_int
        L.orc_solve_masked.argtypes = [yp, gp, dp, dp, dp, dp, dp, C.POINTER(C.c_uint8),
                                       C.c_double, C.c_double, C.c_int, C.c_int64, dp,
                                       C.POINTER(C.c_int64), dp]
        L.orc_query.restype = C.c_int
        L.orc_query.argtypes = [yp, gp, dp, C.c_int, dp, dp, dp, dp, dp, dp]
        L.orc_solve_field.restype = C.c_int
        L.orc_solve_field.argtypes = [yp, gp, dp, dp, dp, dp, dp, C.c_double, C.c_double,
                                      C.c_double, C.c_int, C.c_int64, dp,
                                      C.POINTER(C.c_int64), dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


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
    d.kind = kind
    for i, v in enumerate(params):
        d.p[i] = float(v)
    return d


def _dbounds(dlo, dhi):
    lo = np.zeros(4)
    hi = np.zeros(4)
    if dlo is None or dhi is None:
        return lo, hi
    dlo = np.atleast_1d(np.asarray(dlo, dtype=np.float64))
    dhi = np.atleast_1d(np.asarray(dhi, dtype=np.float64))
    lo[: len(dlo)] = dlo
    hi[: len(dhi)] = dhi
    return lo, hi


def _field(grid: Grid, dfield):
    """Per-node disturbance bounds as the flat (channel, lower/upper, node)
    array the C code takes (None: the constant box is used)."""
    if dfield is None:
        return None, None
    N = int(np.prod([grid.n[i] for i in range(grid.ndim)]))
    f = _f64(dfield).reshape(-1)
    if f.size % (2 * N) != 0:
        raise ValueError("dfield must hold (channels, 2, N) values")
    return f, _dp(f)


def hamiltonian(dyn: Dyn, x, p, dlo, dhi) -> float:
    x = _f64(np.resize(np.asarray(x, dtype=np.float64), 4))
    p = _f64(np.resize(np.asarray(p, dtype=np.float64), 4))
    lo, hi = _dbounds(dlo, dhi)
    return lib().orc_hamiltonian(C.byref(dyn), _dp(x), _dp(p), _dp(lo), _dp(hi))


def dynamics(dyn: Dyn, x, u, d):
    x = _f64(np.resize(np.asarray(x, dtype=np.float64), 4))
    u = _f64(np.resize(np.asarray(u, dtype=np.float64), 4))
    d = _f64(np.resize(np.asarray(d, dtype=np.float64), 4))
    f = np.zeros(4)
    lib().orc_dynamics(C.byref(dyn), _dp(x), _dp(u), _dp(d), _dp(f))
    return f


def lf_alpha(dyn: Dyn, grid: Grid, dlo, dhi, dfield=None):
    lo, hi = _dbounds(dlo, dhi)
    keep, fp = _field(grid, dfield)
    a = np.zeros(4)
    lib().orc_lf_alpha_field(C.byref(dyn), C.byref(grid), _dp(lo), _dp(hi), fp, _dp(a))
    return a[: grid.ndim]


def dt(grid: Grid, alpha, cfl: float = 0.8) -> float:
    a = np.zeros(4)
    a[: len(alpha)] = alpha
    return lib().orc_dt(C.byref(grid), _dp(a), cfl)


def line_derivs(v, h: float, order: int = 2):
    v = _f64(v)
    pm = np.zeros_like(v)
    pp = np.zeros_like(v)
    lib().orc_line_derivs(_dp(v), len(v), h, order, _dp(pm), _dp(pp))
    return pm, pp


def spatial_op(dyn, grid, dlo, dhi, alpha, V, order=2, dfield=None):
    V = _f64(V)
    lo, hi = _dbounds(dlo, dhi)
    keep, fp = _field(grid, dfield)
    a = np.zeros(4)
    a[: len(alpha)] = alpha
    L = np.zeros_like(V)
    lib().orc_spatial_op_field(C.byref(dyn), C.byref(grid), _dp(lo), _dp(hi), fp, _dp(a),
                               order, _dp(V), _dp(L))
    return L


def iterate(dyn, grid, dlo, dhi, alpha, dt_, l, V, order=2, dfield=None):
    V = _f64(V)
    l = _f64(l)
    lo, hi = _dbounds(dlo, dhi)
    keep, fp = _field(grid, dfield)
    a = np.zeros(4)
    a[: len(alpha)] = alpha
    Vn = np.zeros_like(V)
    r = lib().orc_iterate_field(C.byref(dyn), C.byref(grid), _dp(lo), _dp(hi), fp, _dp(a),
                                dt_, order, _dp(l), _dp(V), _dp(Vn))
    return Vn, r


def iterate_at(dyn, grid, dlo, dhi, alpha, dt_, l, V, idx, order=2, dfield=None) -> float:
    V = _f64(V)
    l = _f64(l)
    lo, hi = _dbounds(dlo, dhi)
    keep, fp = _field(grid, dfield)
    a = np.zeros(4)
    a[: len(alpha)] = alpha
    return lib().orc_iterate_at_field(C.byref(dyn), C.byref(grid), _dp(lo), _dp(hi), fp,
                                      _dp(a), dt_, order, _dp(l), _dp(V), int(idx))


def residual_band(V, Vnew, band):
    V, Vnew = _f64(V), _f64(Vnew)
    return lib().orc_residual_band(V.size, _dp(V), _dp(Vnew), float(band))


def solve(dyn, grid, l, dlo, dhi, tol=1e-4, V0=None, cfl=0.8, order=2,
          max_iter=100000, history=False, band=0.0, dfield=None):
    """Returns dict(V, status, iterations, residual, dt, alpha, res_hist, max_rise).
    band > 0 restricts the stop test to nodes with |V| < band before or after
    the step (see orc_residual_band).  dfield: per-node disturbance bounds,
    shape (channels, 2, N) (lower, upper), used instead of dlo/dhi."""
    l = _f64(l)
    lo, hi = _dbounds(dlo, dhi)
    keep, fp = _field(grid, dfield)
    V = np.zeros_like(l)
    it = C.c_int64(0)
    res = C.c_double(0)
    dt_ = C.c_double(0)
    a = np.zeros(4)
    hist = np.zeros(max(int(max_iter), 1)) if history else None
    rise = C.c_double(0)
    v0p = None
    if V0 is not None:
        V0 = _f64(V0)
        v0p = _dp(V0)
    st = lib().orc_solve_field(C.byref(dyn), C.byref(grid), _dp(l), v0p, _dp(lo), _dp(hi),
                               fp, float(tol), float(band), float(cfl), int(order),
                               int(max_iter), _dp(V), C.byref(it), C.byref(res),
                               C.byref(dt_), _dp(a), _dp(hist) if history else None,
                               C.byref(rise))
    out = dict(V=V, status=st, iterations=it.value, residual=res.value, dt=dt_.value,
               alpha=a[: grid.ndim].copy(), max_rise=rise.value)
    if history:
        out["res_hist"] = hist[: it.value].copy()
    return out


def interp(src: Grid, Vs, dst: Grid):
    Vs = _f64(Vs)
    n = [dst.n[i] for i in range(dst.ndim)]
    Vd = np.zeros(int(np.prod(n)))
    st = lib().orc_interp(C.byref(src), _dp(Vs), C.byref(dst), _dp(Vd))
    if st != OK:
        raise ValueError("orc_interp: grids do not share a box")
    return Vd


def refine_mask(grid: Grid, V):
    V = _f64(V)
    nc = [grid.n[i] - 1 for i in range(grid.ndim)]
    m = np.zeros(int(np.prod(nc)), dtype=np.uint8)
    cnt = lib().orc_refine_mask(C.byref(grid), _dp(V),
                                m.ctypes.data_as(C.POINTER(C.c_uint8)))
    return m, int(cnt)


def query(dyn: Dyn, grid: Grid, V, X, dlo, dhi, order=2):
    """Safety query at every row of X (states, shape (n, ndim)): returns
    dict(value (n,), grad (n, ndim), u (n, controls), ok (n,) bool)."""
    V = _f64(V)
    X = np.atleast_2d(_f64(X))
    lo, hi = _dbounds(dlo, dhi)
    D = grid.ndim
    m = 2 if dyn.kind == DI2X2 else 1
    n = X.shape[0]
    val = np.zeros(n)
    grad = np.zeros((n, D))
    u = np.zeros((n, m))
    ok = np.zeros(n, dtype=bool)
    xb, gb, ub, vb = np.zeros(4), np.zeros(4), np.zeros(4), C.c_double(0)
    for i in range(n):
        xb[:D] = X[i]
        st = lib().orc_query(C.byref(dyn), C.byref(grid), _dp(V), int(order), _dp(lo), _dp(hi),
                             _dp(xb), C.byref(vb), _dp(gb), _dp(ub))
        val[i] = vb.value
        grad[i] = gb[:D]
        u[i] = ub[:m]
        ok[i] = st == OK
    return dict(value=val, grad=grad, u=u, ok=ok)


def query_decomposed(subs, X, level=0.0, U_perf=None, order=2):
    """Decomposed query at every row of X (full states).  subs: list of
    dicts with dyn, grid, V, state_index (list), control_index, dlo, dhi.
    Returns dict(value, active, sub_value (n, nsub), grad (n, state_dim),
    u (n, controls), u_out, ok)."""
    X = np.atleast_2d(_f64(X))
    n, dim = X.shape
    ns = len(subs)
    dyns = (Dyn * ns)(*[s["dyn"] for s in subs])
    grids = (Grid * ns)(*[s["grid"] for s in subs])
    Vs = [_f64(s["V"]) for s in subs]
    Vp = (C.POINTER(C.c_double) * ns)(*[_dp(v) for v in Vs])
    sidx = np.zeros(4 * ns, dtype=np.int32)
    for k, sb in enumerate(subs):
        sidx[4 * k: 4 * k + len(sb["state_index"])] = sb["state_index"]
    cidx = np.array([sb["control_index"] for sb in subs], dtype=np.int32)
    m = int(max(sb["control_index"] + (2 if sb["dyn"].kind == DI2X2 else 1) for sb in subs))
    bounds = [_dbounds(sb["dlo"], sb["dhi"]) for sb in subs]
    lo_p = (C.POINTER(C.c_double) * ns)(*[_dp(b[0]) for b in bounds])
    hi_p = (C.POINTER(C.c_double) * ns)(*[_dp(b[1]) for b in bounds])
    U = np.zeros((n, m)) if U_perf is None else np.atleast_2d(_f64(U_perf))
    out = dict(value=np.zeros(n), active=np.zeros(n, dtype=np.int32), sub_value=np.zeros((n, ns)),
               grad=np.zeros((n, dim)), u=np.zeros((n, m)), u_out=np.zeros((n, m)),
               ok=np.zeros(n, dtype=bool))
    v, a = C.c_double(0), C.c_int32(0)
    sv, g, u, uo = np.zeros(ns), np.zeros(dim), np.zeros(m), np.zeros(m)
    ip = C.POINTER(C.c_int32)
    for i in range(n):
        xi = _f64(X[i])
        ui = _f64(U[i])
        st = lib().orc_query_decomposed(ns, dyns, grids, Vp, sidx.ctypes.data_as(ip),
                                        cidx.ctypes.data_as(ip), lo_p, hi_p, int(order), _dp(xi),
                                        float(level), _dp(ui), C.byref(v), C.byref(a), _dp(sv),
                                        _dp(g), _dp(u), _dp(uo))
        out["value"][i], out["active"][i] = v.value, a.value
        out["sub_value"][i], out["grad"][i], out["u"][i], out["u_out"][i] = sv, g, u, uo
        out["ok"][i] = st == OK
    return out


def band_mask(grid: Grid, V, k: int):
    """Nodes within k cells of a cell straddling V = 0 (uint8 array, count)."""
    V = _f64(V)
    m = np.zeros(V.size, dtype=np.uint8)
    cnt = lib().orc_band_mask(C.byref(grid), _dp(V), int(k), m.ctypes.data_as(C.POINTER(C.c_uint8)))
    return m, int(cnt)


def solve_masked(dyn, grid, l, dlo, dhi, mask, tol=1e-4, V0=None, cfl=0.8, order=2,
                 max_iter=100000, dfield=None):
    """Localized solve: only the nodes with mask != 0 are updated."""
    l = _f64(l)
    lo, hi = _dbounds(dlo, dhi)
    keep, fp = _field(grid, dfield)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    V = np.zeros_like(l)
    it = C.c_int64(0)
    res = C.c_double(0)
    v0p = None
    if V0 is not None:
        V0 = _f64(V0)
        v0p = _dp(V0)
    st = lib().orc_solve_masked(C.byref(dyn), C.byref(grid), _dp(l), v0p, _dp(lo), _dp(hi), fp,
                                m.ctypes.data_as(C.POINTER(C.c_uint8)), float(tol), float(cfl),
                                int(order), int(max_iter), _dp(V), C.byref(it), C.byref(res))
    return dict(V=V, status=st, iterations=it.value, residual=res.value)
