"""The allocation-free solve (hjr_solve_device_noalloc) against hjr_solve_device.

Both run the same kernels, so on the same inputs they must give bitwise the same value function,
iteration counts and status.  Two calls in a row, the second on a smaller grid (the static
scratch block keeps the first call's contents, which the second must not rely on), then a
problem too large for the block (refused before any device work) and a small one after it.
"""
import numpy as np
import pytest

from paper_1903_07715_amd import workloads as W

pytestmark = pytest.mark.gpu


def _pair(hjrlib, gpu, p, k=None, stream=None, **extra):
    import torch

    lt = torch.tensor(p.l, device=gpu)
    kt = None if k is None else torch.tensor(k, device=gpu)
    opts = hjrlib.problem_options(p, max_iter=20000, **extra)
    Va = torch.empty_like(lt)
    ra, sa = hjrlib.solve_device(p.grid, p.dyn, lt, kt, Va, **opts)
    Vb = torch.full_like(lt, float("nan"))
    torch.cuda.synchronize()
    rb, sb = hjrlib.solve_device_noalloc(p.grid, p.dyn, lt, kt, Vb, stream=stream, **opts)
    torch.cuda.synchronize()
    print(f"[noalloc] {p.name}: {rb['iterations']}+{rb['polish_iterations']} steps, status {sb}", flush=True)
    assert sa == sb
    assert (ra["iterations"], ra["polish_iterations"]) == (rb["iterations"], rb["polish_iterations"])
    assert torch.equal(Va, Vb)
    return Vb


def test_noalloc_matches_solve_device_twice_then_smaller(gpu, hjrlib):
    import torch

    big = W.dubins_problem(81, dbar=0.1)
    prior = W.dubins_problem(81, dbar=0.05)
    kt = torch.tensor(prior.l, device=gpu)
    K = torch.empty_like(kt)
    hjrlib.solve_device(prior.grid, prior.dyn, kt, None, K,
                        **hjrlib.problem_options(prior, precision=hjrlib.FP64, max_iter=20000))
    k = K.cpu().numpy()
    _pair(hjrlib, gpu, big, k, precision=hjrlib.FP32_POLISH64)         # 531 441 nodes, warm
    small = W.dubins_problem(41, dbar=0.1)
    _pair(hjrlib, gpu, small, precision=hjrlib.FP32_POLISH64)          # 68 921 nodes, cold
    di = W.di_box_problem(101, dbar=0.1)
    s = torch.cuda.Stream()
    _pair(hjrlib, gpu, di, precision=hjrlib.FP64, stream=s)             # FP64 upwind on a caller stream


def test_noalloc_6d_bricks(gpu, hjrlib, monkeypatch):
    """A 6-D quadrotor through the brick plane-march kernel, whose tile list the scratch block
    also has to hold."""
    monkeypatch.setenv("HJR_NPT", "-16")
    _pair(hjrlib, gpu, W.quad6_problem(9), precision=hjrlib.FP32_POLISH64)   # 531 441 nodes


def test_noalloc_refuses_a_grid_beyond_its_block(gpu, hjrlib):
    import torch

    p = W.quad6_problem(13)  # 4.8 M nodes: more than the static block holds
    lt = torch.tensor(p.l, device=gpu)
    V = torch.empty_like(lt)
    with pytest.raises(hjrlib.HJRError) as e:
        hjrlib.solve_device_noalloc(p.grid, p.dyn, lt, None, V, **hjrlib.problem_options(p))
    assert e.value.status == hjrlib.ERR_BUDGET
    _pair(hjrlib, gpu, W.dubins_problem(25), precision=hjrlib.FP32_POLISH64)  # still works afterwards
