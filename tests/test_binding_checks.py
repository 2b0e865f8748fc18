"""The binding rejects device-array arguments the library would misread, before any launch.

Every device entry point takes raw pointers, so a short array, a wrong element type, a strided
view or a host tensor would make its kernels read or write out of bounds.  These checks run on
the CPU: the type, layout and size checks come before the GPU-memory check, so CPU tensors
exercise all of them, and nothing reaches the library.
"""
import pytest
import torch

from paper_1903_07715_amd import hjr
from paper_1903_07715_amd import workloads as W

G = W.Grid((9, 9), (-1, -1), (1, 1))
DYN = W.double_integrator(1.0, 1.0, 0.1)


def _good(n=G.size, dtype=torch.float64):
    return torch.zeros(n, dtype=dtype)


def _bad_cases(n=G.size, dtype=torch.float64):
    other = torch.float32 if dtype == torch.float64 else torch.float64
    return {
        "dtype": torch.zeros(n, dtype=other),
        "int64": torch.zeros(n, dtype=torch.int64),
        "complex": torch.zeros(n, dtype=torch.complex64),
        "short": torch.zeros(n - 1, dtype=dtype),
        "long": torch.zeros(n + 1, dtype=dtype),
        "strided": torch.zeros(2 * n, dtype=dtype)[::2],
        "host": torch.zeros(n, dtype=dtype),  # right in every respect but its device
        "numpy": torch.zeros(n, dtype=dtype).numpy(),
    }


@pytest.mark.parametrize("case", list(_bad_cases()))
@pytest.mark.parametrize("arg", ["l", "k", "V"])
def test_solve_device_rejects_bad_arrays(case, arg):
    args = {"l": _good(), "k": None, "V": _good()}
    args[arg] = _bad_cases()[case]
    with pytest.raises(ValueError):
        hjr.solve_device(G, DYN, args["l"], args["k"], args["V"])


def test_solve_device_rejects_a_bad_constraint():
    with pytest.raises(ValueError):
        hjr.solve_device(G, DYN, _good(), None, _good(), constraint=_good(G.size - 3))


@pytest.mark.parametrize("case", list(_bad_cases(dtype=torch.float32)))
def test_stage_device_rejects_bad_arrays_in_fp32(case):
    bad = _bad_cases(dtype=torch.float32)[case]
    good = _good(dtype=torch.float32)
    for pos in range(4):
        arrs = [good, good, good, good]
        arrs[pos] = bad
        with pytest.raises(ValueError):
            hjr.stage_device(G, DYN, 1, 0.01, *arrs, spatial=hjr.UPWIND1, temporal=hjr.EULER, precision=hjr.FP32)


def test_stage_device_fp64_rejects_fp32_arrays():
    a = _good(dtype=torch.float32)
    with pytest.raises(ValueError):
        hjr.stage_device(G, DYN, 1, 0.01, a, a, a, a, spatial=hjr.UPWIND1, temporal=hjr.EULER, precision=hjr.FP64)


@pytest.mark.parametrize("case", list(_bad_cases()))
def test_context_submit_rejects_bad_arrays(case):
    ctx = hjr.Context.__new__(hjr.Context)  # no device context: the checks come first
    ctx._h = None
    ctx._keep = {}
    for arg in ("l", "k", "V"):
        args = {"l": _good(), "k": _good(), "V": _good()}
        args[arg] = _bad_cases()[case]
        with pytest.raises(ValueError):
            ctx.submit(G, DYN, args["l"], args["k"], args["V"])


@pytest.mark.parametrize("case", list(_bad_cases()))
def test_query_entry_points_reject_bad_arrays(case):
    table_n = (G.ndim + 1) * G.size
    with pytest.raises(ValueError):
        hjr.gradient_device(G, _bad_cases()[case], _good(table_n))
    with pytest.raises(ValueError):
        hjr.gradient_device(G, _good(), _bad_cases(table_n)[case])
    x = torch.zeros((5, 2), dtype=torch.float64)
    with pytest.raises(ValueError):
        hjr.safe_control_device(G, DYN, _bad_cases(table_n)[case], x, _good(5))
    with pytest.raises(ValueError):
        hjr.safe_control_device(G, DYN, _good(table_n), x, _bad_cases(5)[case])
