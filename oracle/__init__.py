"""ctypes front end of the FP64 CPU reference solver (hjr_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import this package; the GPU library never does, and this package imports
nothing from the GPU library (the grid and model records it accepts are plain data from
``paper_1903_07715_amd.workloads``).

The C source is built with gcc on first use (or by ``build()``) into ``oracle/liboracle.so``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hjr_oracle.c")
_HDR = os.path.join(_HERE, "hjr_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

AVOID, REACH = 0, 1
UPWIND1, WENO5 = 1, 5
EULER, RK3 = 1, 3
CONV_STEP, CONV_INTERVAL = 0, 1
MAXD = 6


class _Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * MAXD), ("lo", C.c_double * MAXD),
                ("hi", C.c_double * MAXD), ("periodic", C.c_uint32)]


class _Dyn(C.Structure):
    _fields_ = [("id", C.c_int32), ("n_params", C.c_int32), ("p", C.c_double * 16)]


class _Opts(C.Structure):
    _fields_ = [("game", C.c_int32), ("spatial", C.c_int32), ("temporal", C.c_int32),
                ("conv_mode", C.c_int32), ("min_each_stage", C.c_int32), ("brs", C.c_int32),
                ("cfl", C.c_double), ("tol", C.c_double), ("dt_report", C.c_double),
                ("t_max", C.c_double), ("dt_max", C.c_double), ("max_iter", C.c_int64),
                ("discount", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("steps", C.c_int64), ("intervals", C.c_int64), ("t", C.c_double),
                ("last_delta", C.c_double), ("dt", C.c_double), ("converged", C.c_int32),
                ("pad", C.c_int32), ("discounted_steps", C.c_int64)]


def build(force: bool = False) -> str:
    """Compile hjr_oracle.c with gcc (FP64, no FMA contraction, OpenMP)."""
    with _lock:
        fresh = os.path.exists(_LIB) and os.path.getmtime(_LIB) >= max(
            os.path.getmtime(_SRC), os.path.getmtime(_HDR))
        if fresh and not force:
            return _LIB
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
        return _LIB


def _load():
    global _lib
    if _lib is None:
        # HJR_ORACLE_LIBRARY: load another build of the oracle (a copy with a planted mistake,
        # to check that the pins catch it); otherwise build this one if needed
        alt = os.environ.get("HJR_ORACLE_LIBRARY")
        if not alt:
            build()
        lib = C.CDLL(alt or _LIB)
        P = C.POINTER
        dp = P(C.c_double)
        lib.or_hamiltonian.argtypes = [P(_Dyn), C.c_int, dp, dp, dp, dp]
        lib.or_flow.argtypes = [P(_Dyn), dp, dp, dp, dp]
        lib.or_weno5.argtypes = [C.c_double] * 5
        lib.or_weno5.restype = C.c_double
        lib.or_derivatives.argtypes = [P(_Grid), C.c_int, dp, C.c_int64, C.c_int, dp, dp]
        lib.or_operator.argtypes = [P(_Grid), P(_Dyn), C.c_int, C.c_int, dp, dp]
        lib.or_operator_at.argtypes = [P(_Grid), P(_Dyn), C.c_int, C.c_int, dp, P(C.c_int64), C.c_int64, dp]
        lib.or_stage_at.argtypes = [P(_Grid), P(_Dyn), P(_Opts), C.c_int, C.c_double, dp, dp, dp,
                                    P(C.c_int64), C.c_int64, dp]
        lib.or_cfl_dt.argtypes = [P(_Grid), P(_Dyn), C.c_double, C.c_double]
        lib.or_cfl_dt.restype = C.c_double
        lib.or_step.argtypes = [P(_Grid), P(_Dyn), P(_Opts), dp, dp, C.c_double, dp, dp]
        lib.or_solve.argtypes = [P(_Grid), P(_Dyn), dp, dp, P(_Opts), dp, P(_Result)]
        lib.or_step_ra.argtypes = [P(_Grid), P(_Dyn), P(_Opts), dp, dp, dp, C.c_double, dp, dp]
        lib.or_solve_ra.argtypes = [P(_Grid), P(_Dyn), dp, dp, dp, P(_Opts), dp, P(_Result)]
        lib.or_threads.restype = C.c_int
        lib.or_num_controls.argtypes = [C.c_int]
        lib.or_num_controls.restype = C.c_int
        lib.or_gradient_at.argtypes = [P(_Grid), C.c_int, dp, C.c_int64, dp]
        lib.or_interp_at.argtypes = [P(_Grid), C.c_int, dp, dp, dp, dp]
        lib.or_optimal_control.argtypes = [P(_Dyn), C.c_int, dp, dp, dp]
        lib.or_safe_control.argtypes = [P(_Grid), P(_Dyn), C.c_int, C.c_int, dp, dp, C.c_int64, dp, dp, dp]
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().or_threads())


def _grid(g) -> _Grid:
    s = _Grid()
    s.ndim = g.ndim
    for i in range(g.ndim):
        s.n[i] = g.n[i]
        s.lo[i] = g.lo[i]
        s.hi[i] = g.hi[i]
    s.periodic = g.periodic_mask
    return s


def _dyn(d) -> _Dyn:
    s = _Dyn()
    s.id = d.id
    s.n_params = len(d.params)
    for i, v in enumerate(d.params):
        s.p[i] = v
    return s


def _opts(spatial=UPWIND1, temporal=EULER, game=AVOID, cfl=0.8, tol=1e-6, conv_mode=CONV_STEP,
          dt_report=0.01, t_max=0.0, dt_max=0.0, max_iter=200000, min_each_stage=False, brs=False,
          discount=0.0) -> _Opts:
    o = _Opts()
    o.game, o.spatial, o.temporal, o.conv_mode = game, spatial, temporal, conv_mode
    o.min_each_stage = int(bool(min_each_stage))
    o.brs = int(bool(brs))
    o.discount = discount
    o.cfl, o.tol, o.dt_report, o.t_max, o.dt_max, o.max_iter = cfl, tol, dt_report, t_max, dt_max, max_iter
    return o


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def hamiltonian(dyn, x, p, game=AVOID):
    """H(x, p) (eq. (6)) and the dissipation coefficients alpha_i(x)."""
    x = _f64(x)
    p = _f64(p)
    H = C.c_double()
    alpha = np.zeros(dyn.ndim)
    rc = _load().or_hamiltonian(C.byref(_dyn(dyn)), game, _ptr(x), _ptr(p), C.byref(H), _ptr(alpha))
    if rc:
        raise ValueError("or_hamiltonian failed")
    return H.value, alpha


def flow(dyn, x, u, d):
    f = np.zeros(dyn.ndim)
    u = _f64(np.resize(np.asarray(u, dtype=np.float64), 3))
    d = _f64(np.resize(np.asarray(d, dtype=np.float64), 3))
    _load().or_flow(C.byref(_dyn(dyn)), _ptr(_f64(x)), _ptr(u), _ptr(d), _ptr(f))
    return f


def weno5(v1, v2, v3, v4, v5) -> float:
    return float(_load().or_weno5(v1, v2, v3, v4, v5))


def derivatives(grid, V, node, dim, spatial=WENO5):
    V = _f64(V)
    dm, dp = C.c_double(), C.c_double()
    rc = _load().or_derivatives(C.byref(_grid(grid)), spatial, _ptr(V), int(node), dim, C.byref(dm), C.byref(dp))
    if rc:
        raise ValueError("or_derivatives failed")
    return dm.value, dp.value


def operator(grid, dyn, V, spatial=WENO5, game=AVOID) -> np.ndarray:
    """L(V) = H(x, (D- + D+)/2) + sum_i alpha_i (D+ - D-)/2 at every node."""
    V = _f64(V)
    L = np.empty_like(V)
    if _load().or_operator(C.byref(_grid(grid)), C.byref(_dyn(dyn)), game, spatial, _ptr(V), _ptr(L)):
        raise ValueError("or_operator failed")
    return L


def operator_at(grid, dyn, V, nodes, spatial=WENO5, game=AVOID) -> np.ndarray:
    V = _f64(V)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.empty(nodes.shape[0])
    rc = _load().or_operator_at(C.byref(_grid(grid)), C.byref(_dyn(dyn)), game, spatial, _ptr(V),
                                nodes.ctypes.data_as(C.POINTER(C.c_int64)), nodes.shape[0], _ptr(out))
    if rc:
        raise ValueError("or_operator_at failed")
    return out


def stage_at(grid, dyn, stage, dt, Vs, Vn, l, nodes, **opts) -> np.ndarray:
    """One time-integrator stage evaluated at the given flat node indices."""
    Vs, Vn, l = _f64(Vs), _f64(Vn), _f64(l)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.empty(nodes.shape[0])
    o = _opts(**opts)
    rc = _load().or_stage_at(C.byref(_grid(grid)), C.byref(_dyn(dyn)), C.byref(o), stage, dt, _ptr(Vs), _ptr(Vn),
                             _ptr(l), nodes.ctypes.data_as(C.POINTER(C.c_int64)), nodes.shape[0], _ptr(out))
    if rc:
        raise ValueError("or_stage_at failed")
    return out


def cfl_dt(grid, dyn, cfl=0.8, dt_max=0.0) -> float:
    dt = _load().or_cfl_dt(C.byref(_grid(grid)), C.byref(_dyn(dyn)), cfl, dt_max)
    if dt < 0:
        raise ValueError("or_cfl_dt failed")
    return float(dt)


def step(grid, dyn, V, l, dt, constraint=None, **opts):
    """One full time step: returns (V_next, max |V_next - V|).  constraint: the reach-avoid
    constraint function g (the step then ends with max(g, .))."""
    V, l = _f64(V), _f64(l)
    gc = None if constraint is None else _f64(constraint, V.shape)
    out = np.empty_like(V)
    delta = C.c_double()
    o = _opts(**opts)
    if _load().or_step_ra(C.byref(_grid(grid)), C.byref(_dyn(dyn)), C.byref(o), _ptr(l),
                          None if gc is None else _ptr(gc), _ptr(V), dt, _ptr(out), C.byref(delta)):
        raise ValueError("or_step failed")
    return out, delta.value


def solve(grid, dyn, l, k=None, constraint=None, **opts):
    """Iterate to convergence from l (k is None) or from min(k, l); with a reach-avoid
    constraint function g, from max(g, .) with max(g, .) after every step.  Returns (V, info)."""
    l = _f64(l, grid.shape)
    kk = None if k is None else _f64(k, grid.shape)
    gc = None if constraint is None else _f64(constraint, grid.shape)
    V = np.empty(grid.shape)
    res = _Result()
    o = _opts(**opts)
    rc = _load().or_solve_ra(C.byref(_grid(grid)), C.byref(_dyn(dyn)), _ptr(l), None if gc is None else _ptr(gc),
                             None if kk is None else _ptr(kk), C.byref(o), _ptr(V), C.byref(res))
    if rc == -3:
        raise FloatingPointError("non-finite input")
    if rc:
        raise ValueError(f"or_solve failed ({rc})")
    info = dict(steps=res.steps, intervals=res.intervals, t=res.t, last_delta=res.last_delta, dt=res.dt,
                converged=res.converged, discounted_steps=res.discounted_steps)
    return V, info


def problem_opts(problem) -> dict:
    """Scheme options of a workloads.Problem."""
    return dict(spatial=problem.spatial, temporal=problem.temporal, game=problem.game, cfl=problem.cfl,
                tol=problem.tol)


def num_controls(dyn) -> int:
    return int(_load().or_num_controls(dyn.id))


def gradient_at(grid, V, nodes, spatial=UPWIND1) -> np.ndarray:
    """Nodal gradient (D- + D+)/2 at the given flat nodes: array (len(nodes), ndim)."""
    V = _f64(V)
    if V.size != grid.size:
        raise ValueError("V does not match the grid")
    nodes = np.asarray(nodes, dtype=np.int64).ravel()
    out = np.empty((nodes.shape[0], grid.ndim))
    g = _grid(grid)
    lib = _load()
    for i, nd in enumerate(nodes):
        row = np.empty(grid.ndim)
        if lib.or_gradient_at(C.byref(g), spatial, _ptr(V), int(nd), _ptr(row)):
            raise ValueError("or_gradient_at failed")
        out[i] = row
    return out


def optimal_control(dyn, x, p, game=AVOID) -> np.ndarray:
    u = np.zeros(3)
    if _load().or_optimal_control(C.byref(_dyn(dyn)), game, _ptr(_f64(x)), _ptr(_f64(p)), _ptr(u)):
        raise ValueError("or_optimal_control failed")
    return u[: num_controls(dyn)].copy()


def safe_control(grid, dyn, V, x, game=AVOID, spatial=UPWIND1):
    """Safe control at states x (nq x ndim): returns (u (nq x nu), p (nq x ndim), v (nq))."""
    V = _f64(V)
    if V.size != grid.size:
        raise ValueError("V does not match the grid")
    x = _f64(x).reshape(-1, grid.ndim)
    nq = x.shape[0]
    nu = num_controls(dyn)
    u = np.empty((nq, nu))
    p = np.empty((nq, grid.ndim))
    v = np.empty(nq)
    rc = _load().or_safe_control(C.byref(_grid(grid)), C.byref(_dyn(dyn)), game, spatial, _ptr(V), _ptr(x), nq,
                                 _ptr(u), _ptr(p), _ptr(v))
    if rc:
        raise ValueError("or_safe_control failed")
    return u, p, v
