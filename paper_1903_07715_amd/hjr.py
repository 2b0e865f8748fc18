"""Thin ctypes binding of libhjr (include/hjr.h): argument marshalling only.

Every computation runs in the gfx950 kernels of libhjr.so.  There is no CPU fallback: if the
library is missing, ``load()`` raises.  PyTorch is used only to hand device memory and streams
to the library (``solve_device``, ``stage_device``, ``Context.submit``).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HJR_LIBRARY") or os.path.join(_HERE, "libhjr.so")
MAX_DIM = 6
MAX_PARAMS = 16

OK, NOT_CONVERGED, PENDING, HORIZON = 0, 1, 2, 3
ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_NONFINITE, ERR_OOM, ERR_DEVICE, ERR_BUDGET, ERR_UNKNOWN_TICKET = (
    -1, -2, -3, -4, -5, -6, -7)
AVOID, REACH = 0, 1
UPWIND1, WENO5 = 1, 5
EULER, TVDRK3 = 1, 3
FP64, FP32, FP32_POLISH64 = 0, 1, 2
CONV_PER_STEP, CONV_PER_INTERVAL = 0, 1

EXPORTED = ["hjr_abi_version", "hjr_build_id", "hjr_default_options", "hjr_status_string", "hjr_last_error",
            "hjr_device_count", "hjr_solve", "hjr_solve_device", "hjr_solve_device_noalloc", "hjr_batch_solve",
            "hjr_cfl_dt",
            "hjr_stage_device", "hjr_ctx_create", "hjr_submit", "hjr_poll", "hjr_ctx_drain",
            "hjr_ctx_get_stats", "hjr_ctx_destroy", "hjr_profile_enable", "hjr_profile_read",
            "hjr_num_controls", "hjr_gradient_device", "hjr_safe_control_device", "hjr_solve_reach_avoid",
            "hjr_solve_reach_avoid_device", "hjr_local_dependencies", "hjr_march_plan"]


class Grid_(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * MAX_DIM), ("lo", C.c_double * MAX_DIM),
                ("hi", C.c_double * MAX_DIM), ("periodic_mask", C.c_uint32)]


class Dynamics_(C.Structure):
    _fields_ = [("id", C.c_int32), ("n_params", C.c_int32), ("params", C.c_double * MAX_PARAMS)]


class Options_(C.Structure):
    _fields_ = [("game", C.c_int32), ("spatial", C.c_int32), ("temporal", C.c_int32),
                ("precision", C.c_int32), ("conv_mode", C.c_int32), ("steps_per_sync", C.c_int32),
                ("cfl", C.c_double), ("tol", C.c_double), ("tol_fp32", C.c_double),
                ("polish_shift", C.c_double), ("dt_report", C.c_double), ("t_max", C.c_double),
                ("dt_max", C.c_double), ("max_iter", C.c_int64), ("stall_window", C.c_int64),
                ("brs", C.c_int32), ("local_updates", C.c_int32), ("discount", C.c_double)]


class Result_(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("polish_iterations", C.c_int64), ("intervals", C.c_int64),
                ("t_final", C.c_double), ("last_delta", C.c_double), ("dt", C.c_double),
                ("max_abs_l", C.c_double), ("seconds", C.c_double), ("converged", C.c_int32),
                ("pad", C.c_int32), ("discounted_iterations", C.c_int64), ("node_updates", C.c_int64)]


class Problem_(C.Structure):
    _fields_ = [("grid", Grid_), ("dyn", Dynamics_), ("opts", Options_), ("l", C.POINTER(C.c_double)),
                ("k", C.POINTER(C.c_double)), ("V_out", C.POINTER(C.c_double)), ("result", Result_),
                ("status", C.c_int32), ("pad", C.c_int32)]


class CtxStats_(C.Structure):
    _fields_ = [("admitted", C.c_int64), ("finished", C.c_int64), ("queued", C.c_int64),
                ("running", C.c_int64), ("bytes_in_use", C.c_int64), ("bytes_peak", C.c_int64),
                ("budget", C.c_int64), ("chunks", C.c_int64), ("launches", C.c_int64)]


class KernelTime_(C.Structure):
    _fields_ = [("launches", C.c_int64), ("nodes", C.c_int64), ("ms", C.c_double), ("working_launches", C.c_int64),
                ("working_ms", C.c_double)]


class Profile_(C.Structure):
    _fields_ = [("stage32", KernelTime_ * 3), ("stage64", KernelTime_ * 3)]


class HJRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def load():
    """Load libhjr.so.  Raises if it has not been built: there is no other implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_1903_07715_amd.build`")
        # One HIP runtime per process: PyTorch ships its own libamdhip64 with the same soname, so
        # it is loaded first and libhjr binds to it (loading ours first would hand PyTorch a
        # runtime it was not built against).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        dp = P(C.c_double)
        lib.hjr_abi_version.restype = C.c_int32
        lib.hjr_build_id.restype = C.c_char_p
        lib.hjr_default_options.argtypes = [P(Options_)]
        lib.hjr_status_string.restype = C.c_char_p
        lib.hjr_status_string.argtypes = [C.c_int32]
        lib.hjr_last_error.restype = C.c_char_p
        lib.hjr_device_count.restype = C.c_int32
        lib.hjr_num_controls.restype = C.c_int32
        lib.hjr_solve.argtypes = [P(Grid_), P(Dynamics_), dp, dp, P(Options_), dp, P(Result_)]
        lib.hjr_solve_device.argtypes = [P(Grid_), P(Dynamics_), vp, vp, P(Options_), vp, vp, P(Result_)]
        lib.hjr_solve_device_noalloc.argtypes = [P(Grid_), P(Dynamics_), vp, vp, P(Options_), vp, vp, P(Result_)]
        lib.hjr_solve_reach_avoid.argtypes = [P(Grid_), P(Dynamics_), dp, dp, dp, P(Options_), dp, P(Result_)]
        lib.hjr_solve_reach_avoid_device.argtypes = [P(Grid_), P(Dynamics_), vp, vp, vp, P(Options_), vp, vp,
                                                     P(Result_)]
        lib.hjr_batch_solve.argtypes = [C.c_int32, P(Problem_)]
        lib.hjr_local_dependencies.argtypes = [P(Grid_), C.c_int32, P(C.c_int64), P(C.c_int64), vp, vp]
        lib.hjr_cfl_dt.argtypes = [P(Grid_), P(Dynamics_), C.c_double, C.c_double, dp]
        lib.hjr_march_plan.argtypes = [P(Grid_), C.c_int32, P(C.c_int64), C.c_int64]
        lib.hjr_stage_device.argtypes = [P(Grid_), P(Dynamics_), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                         C.c_int32, C.c_double, vp, vp, vp, vp, dp, vp]
        lib.hjr_ctx_create.argtypes = [C.c_int32, C.c_size_t, P(vp)]
        lib.hjr_submit.argtypes = [vp, P(Grid_), P(Dynamics_), vp, vp, P(Options_), vp, P(C.c_int64)]
        lib.hjr_poll.argtypes = [vp, C.c_int64, P(Result_)]
        lib.hjr_ctx_drain.argtypes = [vp]
        lib.hjr_ctx_get_stats.argtypes = [vp, P(CtxStats_)]
        lib.hjr_ctx_destroy.argtypes = [vp]
        lib.hjr_profile_enable.argtypes = [C.c_int32]
        lib.hjr_profile_read.argtypes = [P(Profile_), C.c_int32]
        lib.hjr_num_controls.argtypes = [C.c_int32]
        lib.hjr_gradient_device.argtypes = [P(Grid_), C.c_int32, vp, vp, vp]
        lib.hjr_safe_control_device.argtypes = [P(Grid_), P(Dynamics_), C.c_int32, vp, vp, C.c_int64, vp, vp, vp,
                                                vp]
        for name in EXPORTED:
            if name not in ("hjr_status_string", "hjr_last_error", "hjr_abi_version", "hjr_build_id", "hjr_device_count",
                            "hjr_num_controls", "hjr_march_plan"):
                getattr(lib, name).restype = C.c_int32
        lib.hjr_march_plan.restype = C.c_int64
        _lib = lib
    return _lib


def last_error() -> str:
    return load().hjr_last_error().decode()


def _check(status: int, allow=(OK, NOT_CONVERGED, HORIZON)) -> int:
    if status not in allow:
        raise HJRError(status, last_error() or load().hjr_status_string(status).decode())
    return status


# --------------------------------------------------------------------------------------------
# Marshalling of the plain-data records in workloads.py
# --------------------------------------------------------------------------------------------

def grid_struct(g) -> Grid_:
    s = Grid_()
    s.ndim = g.ndim
    for i in range(g.ndim):
        s.n[i], s.lo[i], s.hi[i] = g.n[i], g.lo[i], g.hi[i]
    s.periodic_mask = g.periodic_mask
    return s


def dyn_struct(d) -> Dynamics_:
    s = Dynamics_()
    s.id = d.id
    s.n_params = len(d.params)
    for i, v in enumerate(d.params):
        s.params[i] = v
    return s


def options(**kw) -> Options_:
    """Library defaults (hjr_default_options) overridden by keyword arguments."""
    o = Options_()
    _check(load().hjr_default_options(C.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def problem_options(problem, **kw) -> dict:
    """Scheme options of a workloads.Problem as keyword arguments for `options`."""
    d = dict(spatial=problem.spatial, temporal=problem.temporal, game=problem.game, cfl=problem.cfl,
             tol=problem.tol)
    d.update(kw)
    return d


def result_dict(r: Result_) -> dict:
    return {f: getattr(r, f) for f, _ in Result_._fields_ if f != "pad"}


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# --------------------------------------------------------------------------------------------
# Entry points
# --------------------------------------------------------------------------------------------

def abi_version() -> int:
    return int(load().hjr_abi_version())


def build_id() -> str:
    """The source hash compiled into the loaded library (see build.source_hash)."""
    return load().hjr_build_id().decode()


def device_count() -> int:
    return int(load().hjr_device_count())


def solve(grid, dyn, l: np.ndarray, k: Optional[np.ndarray] = None, constraint: Optional[np.ndarray] = None,
          **opts):
    """hjr_solve with host arrays (hjr_solve_reach_avoid when a constraint function g is given).
    Returns (V, result dict, status)."""
    l = np.ascontiguousarray(l, dtype=np.float64).reshape(grid.shape)
    kk = None if k is None else np.ascontiguousarray(k, dtype=np.float64).reshape(grid.shape)
    V = np.empty(grid.shape, dtype=np.float64)
    res = Result_()
    o = options(**opts)
    gs, ds = C.byref(grid_struct(grid)), C.byref(dyn_struct(dyn))
    kp = None if kk is None else _dptr(kk)
    if constraint is None:
        st = load().hjr_solve(gs, ds, _dptr(l), kp, C.byref(o), _dptr(V), C.byref(res))
    else:
        gc = np.ascontiguousarray(constraint, dtype=np.float64).reshape(grid.shape)
        st = load().hjr_solve_reach_avoid(gs, ds, _dptr(l), _dptr(gc), kp, C.byref(o), _dptr(V), C.byref(res))
    _check(st)
    return V, result_dict(res), st


def _device_array(t, name: str, numel: int, dtype: str = "float64", optional: bool = False):
    """Check a torch tensor handed to a device entry point before anything is launched: the
    element type, contiguity and element count the library will assume, and that it lives in
    GPU memory.  Raises ValueError otherwise (a short or host array would make the kernels read
    or write out of bounds)."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name}: a device array is required")
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != getattr(torch, dtype):
        raise ValueError(f"{name}: dtype {t.dtype}, expected torch.{dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: the tensor must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    if not t.is_cuda:
        raise ValueError(f"{name}: the tensor must be in GPU memory")
    return t


def _tptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    return int(getattr(stream, "cuda_stream", stream))


def solve_device(grid, dyn, l_dev, k_dev, V_dev, stream=None, constraint=None, **opts):
    """hjr_solve_device on torch FP64 device tensors (hjr_solve_reach_avoid_device when a
    constraint function g is given as a device tensor).  Returns (result dict, status)."""
    n = grid.size
    _device_array(l_dev, "l", n)
    _device_array(k_dev, "k", n, optional=True)
    _device_array(V_dev, "V", n)
    _device_array(constraint, "constraint", n, optional=True)
    res = Result_()
    o = options(**opts)
    gs, ds = C.byref(grid_struct(grid)), C.byref(dyn_struct(dyn))
    if constraint is None:
        st = load().hjr_solve_device(gs, ds, _tptr(l_dev), _tptr(k_dev), C.byref(o), _tptr(V_dev),
                                     _stream_ptr(stream), C.byref(res))
    else:
        st = load().hjr_solve_reach_avoid_device(gs, ds, _tptr(l_dev), _tptr(constraint), _tptr(k_dev), C.byref(o),
                                                 _tptr(V_dev), _stream_ptr(stream), C.byref(res))
    _check(st)
    return result_dict(res), st


def solve_device_noalloc(grid, dyn, l_dev, k_dev, V_dev, stream=None, **opts):
    """hjr_solve_device_noalloc: hjr_solve_device on torch FP64 device tensors without any
    device allocation (the library's static scratch block; see include/hjr.h for the limit).
    Returns (result dict, status)."""
    n = grid.size
    _device_array(l_dev, "l", n)
    _device_array(k_dev, "k", n, optional=True)
    _device_array(V_dev, "V", n)
    res = Result_()
    o = options(**opts)
    st = load().hjr_solve_device_noalloc(C.byref(grid_struct(grid)), C.byref(dyn_struct(dyn)), _tptr(l_dev),
                                         _tptr(k_dev), C.byref(o), _tptr(V_dev), _stream_ptr(stream), C.byref(res))
    _check(st)
    return result_dict(res), st


def batch_solve(problems: Sequence, ls: Sequence[np.ndarray], ks: Sequence[Optional[np.ndarray]], opts_list):
    """hjr_batch_solve.  problems: (grid, dyn) pairs; opts_list: per-problem option dicts.
    Returns (list of V, list of result dicts, list of statuses)."""
    n = len(problems)
    arr = (Problem_ * n)()
    keep = []
    outs = []
    for i, ((g, d), l, k, od) in enumerate(zip(problems, ls, ks, opts_list)):
        p = arr[i]
        p.grid = grid_struct(g)
        p.dyn = dyn_struct(d)
        p.opts = options(**od)
        la = np.ascontiguousarray(l, dtype=np.float64).reshape(g.shape)
        ka = None if k is None else np.ascontiguousarray(k, dtype=np.float64).reshape(g.shape)
        V = np.empty(g.shape, dtype=np.float64)
        keep += [la, ka]
        outs.append(V)
        p.l = _dptr(la)
        p.k = _dptr(ka) if ka is not None else C.POINTER(C.c_double)()
        p.V_out = _dptr(V)
    st = load().hjr_batch_solve(n, arr)
    if st < 0:
        raise HJRError(st, last_error())
    return outs, [result_dict(arr[i].result) for i in range(n)], [int(arr[i].status) for i in range(n)]


def local_dependencies(grid, reach: int):
    """hjr_local_dependencies: (off, dep) uint32 arrays of the block dependency lists."""
    nb, nd = C.c_int64(), C.c_int64()
    gs = grid_struct(grid)
    _check(load().hjr_local_dependencies(C.byref(gs), reach, C.byref(nb), C.byref(nd), None, None))
    off = np.empty(nb.value + 1, dtype=np.uint32)
    dep = np.empty(max(nd.value, 1), dtype=np.uint32)
    _check(load().hjr_local_dependencies(C.byref(gs), reach, C.byref(nb), C.byref(nd), off.ctypes.data, dep.ctypes.data))
    return off, dep[:nd.value]


def march_plan(grid, config: int) -> np.ndarray:
    """hjr_march_plan: the march tiles for `grid` under launch configuration `config`, in launch
    order, as an int64 array of rows (first column, first plane, planes, columns, rows)."""
    gs = grid_struct(grid)
    n = load().hjr_march_plan(C.byref(gs), config, None, 0)
    if n < 0:
        _check(int(n))
    out = np.zeros((max(n, 1), 5), dtype=np.int64)
    m = load().hjr_march_plan(C.byref(gs), config, out.ctypes.data_as(C.POINTER(C.c_int64)), n)
    if m != n:
        raise HJRError(ERR_INVALID_ARG, "march plan changed between calls")
    return out[:n]


def cfl_dt(grid, dyn, cfl=0.5, dt_max=0.0) -> float:
    out = C.c_double()
    _check(load().hjr_cfl_dt(C.byref(grid_struct(grid)), C.byref(dyn_struct(dyn)), cfl, dt_max, C.byref(out)))
    return out.value


def stage_device(grid, dyn, stage, dt, Vs, Vn, l, out, game=AVOID, spatial=WENO5, temporal=TVDRK3,
                 precision=FP64, stream=None):
    """One integrator stage with the solver's own kernel (torch device tensors of the precision's
    element type).  Returns max |out - Vn| for the step's last stage, else None."""
    dt_name = "float32" if precision == FP32 else "float64"
    for t, name in ((Vs, "Vs"), (Vn, "Vn"), (l, "l"), (out, "out")):
        _device_array(t, name, grid.size, dt_name)
    delta = C.c_double(float("nan"))
    st = load().hjr_stage_device(C.byref(grid_struct(grid)), C.byref(dyn_struct(dyn)), game, spatial, temporal,
                                 stage, precision, dt, _tptr(Vs), _tptr(Vn), _tptr(l), _tptr(out),
                                 C.byref(delta), _stream_ptr(stream))
    _check(st)
    last = temporal == EULER or stage == 3
    return delta.value if last else None


def num_controls(dyn) -> int:
    return int(load().hjr_num_controls(dyn.id))


def gradient_device(grid, V, table, spatial=WENO5, stream=None) -> None:
    """hjr_gradient_device: query table (npts x (ndim + 1): gradient components, then V) of V."""
    _device_array(V, "V", grid.size)
    _device_array(table, "table", (grid.ndim + 1) * grid.size)
    _check(load().hjr_gradient_device(C.byref(grid_struct(grid)), spatial, _tptr(V), _tptr(table),
                                      _stream_ptr(stream)))


def safe_control_device(grid, dyn, table, x, u, p=None, v=None, game=AVOID, stream=None) -> None:
    """hjr_safe_control_device on device tensors: x (nq x ndim) -> u (nq x nu), optional p, v."""
    import torch

    if not isinstance(x, torch.Tensor):
        raise ValueError("x: expected a torch tensor")
    nq = x.shape[0] if x.dim() > 1 else x.numel() // grid.ndim
    _device_array(table, "table", (grid.ndim + 1) * grid.size)
    _device_array(x, "x", nq * grid.ndim)
    _device_array(u, "u", nq * num_controls(dyn))
    _device_array(p, "p", nq * grid.ndim, optional=True)
    _device_array(v, "v", nq, optional=True)
    _check(load().hjr_safe_control_device(C.byref(grid_struct(grid)), C.byref(dyn_struct(dyn)), game, _tptr(table),
                                          _tptr(x), nq, _tptr(u), _tptr(p), _tptr(v), _stream_ptr(stream)))


def profile_enable(on: bool = True) -> None:
    _check(load().hjr_profile_enable(1 if on else 0))


def profile_read(reset: bool = False) -> dict:
    """Stage-kernel launch counts, covered nodes and event-timed milliseconds since the last reset,
    in total and over working launches only (steps some instance of the group was still taking)."""
    p = Profile_()
    _check(load().hjr_profile_read(C.byref(p), 1 if reset else 0))
    out = {}
    for prec in ("stage32", "stage64"):
        arr = getattr(p, prec)
        out[prec] = [dict(launches=arr[i].launches, nodes=arr[i].nodes, ms=arr[i].ms,
                          working_launches=arr[i].working_launches, working_ms=arr[i].working_ms)
                     for i in range(3)]
    return out


class Context:
    """Serving context (hjr_ctx): continuous batching of solves on device arrays."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = C.c_void_p()
        _check(load().hjr_ctx_create(device, budget_bytes, C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, grid, dyn, l_dev, k_dev, V_dev, **opts) -> int:
        n = grid.size
        _device_array(l_dev, "l", n)
        _device_array(k_dev, "k", n, optional=True)
        _device_array(V_dev, "V", n)
        t = C.c_int64()
        o = options(**opts)
        _check(load().hjr_submit(self._h, C.byref(grid_struct(grid)), C.byref(dyn_struct(dyn)), _tptr(l_dev),
                                 _tptr(k_dev), C.byref(o), _tptr(V_dev), C.byref(t)))
        self._keep[t.value] = (l_dev, k_dev, V_dev)
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (status, result dict)."""
        res = Result_()
        st = load().hjr_poll(self._h, ticket, C.byref(res))
        if st == PENDING:
            return None
        self._keep.pop(ticket, None)
        if st == ERR_UNKNOWN_TICKET:
            raise HJRError(st, last_error())
        return st, result_dict(res)

    def drain(self) -> int:
        return _check(load().hjr_ctx_drain(self._h))

    def stats(self) -> dict:
        s = CtxStats_()
        _check(load().hjr_ctx_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in CtxStats_._fields_}

    def close(self):
        if self._h:
            st = load().hjr_ctx_destroy(self._h)
            self._h = None
            self._keep.clear()
            _check(st)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
