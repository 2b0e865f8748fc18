"""GPU tests of local updates (the exact narrow band): with `local_updates` a step recomputes
only the node blocks whose stencil reach changed in the previous step; every result must be
bitwise the full update's, with the same step counts, while fewer grid points are computed."""
import math

import numpy as np
import pytest

from paper_1903_07715_amd import workloads as W

pytestmark = pytest.mark.gpu


def _both(hjrlib, grid, dyn, l, k=None, constraint=None, **opts):
    full = hjrlib.solve(grid, dyn, l, k, constraint=constraint, **opts)
    loc = hjrlib.solve(grid, dyn, l, k, constraint=constraint, local_updates=1, **opts)
    return full, loc


def _same(full, loc):
    (Vf, rf, sf), (Vl, rl, sl) = full, loc
    assert sf == sl
    for key in ("iterations", "polish_iterations", "intervals", "discounted_iterations", "converged"):
        assert rf[key] == rl[key], key
    assert np.array_equal(Vf, Vl)
    assert 0 < rl["node_updates"] <= rf["node_updates"]
    return rl["node_updates"] / rf["node_updates"]


def test_new_obstacle_is_updated_locally(gpu, hjrlib):
    """Sec. VII's local change: a small obstacle appears beside the Dubins car's; warm-started
    from the old value function, only the region it affects moves."""
    p = W.dubins_problem(41)
    V0, r0, st = hjrlib.solve(p.grid, p.dyn, p.l, None, **hjrlib.problem_options(p))
    assert st == hjrlib.OK
    l2 = np.minimum(p.l, W.disk_sdf(p.grid, (3.0, 3.0), 0.5))
    print("[local] new obstacle, 41^3 Dubins", flush=True)
    frac = _same(*_both(hjrlib, p.grid, p.dyn, l2, V0, **hjrlib.problem_options(p)))
    print(f"[local] computed fraction {frac:.3f}", flush=True)


def test_new_obstacle_double_integrator_skips_blocks(gpu, hjrlib):
    """The same on the 401^2 double integrator (upwind + Euler, FP64: a reach of one node), where
    the new obstacle's influence stays in a small part of the grid's 158 blocks."""
    p = W.di_box_problem(401, ubar=1.0, dbar=0.1)
    opts = dict(spatial=1, temporal=1, cfl=0.8, tol=1e-6, precision=0)
    V0, _, st = hjrlib.solve(p.grid, p.dyn, p.l, None, **opts)
    assert st == hjrlib.OK
    l2 = np.minimum(p.l, W.box_sdf(p.grid, (0.6, 0.6), (0.05, 0.05)))
    frac = _same(*_both(hjrlib, p.grid, p.dyn, l2, V0, **opts))
    print(f"[local] computed fraction {frac:.3f}", flush=True)
    assert frac < 0.8


@pytest.mark.parametrize("precision", ["FP32_POLISH64", "FP32", "FP64"])
def test_dubins_warm_start_bitwise(gpu, hjrlib, precision):
    p = W.dubins_problem(31, dbar=0.1)
    q = W.dubins_problem(31, dbar=0.05)
    k, _, _ = hjrlib.solve(q.grid, q.dyn, q.l, None, **hjrlib.problem_options(q, precision=hjrlib.FP64))
    print(f"[local] dubins warm {precision}", flush=True)
    _same(*_both(hjrlib, p.grid, p.dyn, p.l, k, **hjrlib.problem_options(p, precision=getattr(hjrlib, precision))))


def _periodic_di(n=41):
    g = W.Grid((n, n), (-1.0, -1.0), (1.0, 1.0), (True, True))
    return g, W.double_integrator(1.0, 1.0, 0.1), W.box_sdf(g, (0.0, 0.0), (0.2, 0.2))


@pytest.mark.parametrize("extra", [
    dict(),
    dict(conv_mode=1, dt_report=0.05),
    dict(discount=0.9),
    dict(t_max=0.7, game=1),
    dict(precision=2, discount=0.95, conv_mode=1, dt_report=0.03),
    dict(t_max=0.7, game=1, brs=1),
    dict(precision=1, conv_mode=1, dt_report=0.05, game=1),
], ids=["plain", "interval", "discount", "horizon", "polish-discount-interval", "reachable-set", "fp32-interval"])
def test_euler_double_integrator_modes_bitwise(gpu, hjrlib, extra):
    """Euler ping-pong buffers, interval ends and horizon cuts (step size changes), the
    discount's anneal and the polish hand-over (full steps), on a 181^2 grid (32 blocks)."""
    g = W.Grid((181, 181), (-1.0, -1.0), (1.0, 1.0), (True, True))
    dyn = W.double_integrator(1.0, 1.0, 0.1)
    l = W.box_sdf(g, (0.0, 0.0), (0.2, 0.2))
    opts = dict(spatial=1, temporal=1, cfl=0.8, tol=1e-6, precision=0, max_iter=20000)
    opts.update(extra)
    print(f"[local] DI {extra}", flush=True)
    _same(*_both(hjrlib, g, dyn, l, None, **opts))


def test_reach_avoid_bitwise(gpu, hjrlib):
    g, dyn, l = _periodic_di(121)
    gc = -W.box_sdf(g, (-0.5, 0.0), (0.1, 0.6))
    print("[local] reach-avoid", flush=True)
    _same(*_both(hjrlib, g, dyn, l, None, constraint=gc, spatial=1, temporal=1, cfl=0.8, tol=1e-6, game=1,
                 precision=0))


@pytest.mark.parametrize("env", [{"HJR_NPT": "1"}, {"HJR_NPT": "8"}, {"HJR_FUSED": "1"}, {"HJR_GRAPHS": "1"},
                                 {"HJR_MAX_BLOCKS": "64"}],
                         ids=lambda e: ",".join(f"{k}={v}" for k, v in e.items()))
def test_launch_configurations_bitwise(gpu, hjrlib, monkeypatch, env):
    """Tiles smaller and larger than a block, the fused kernel, graph replay and a persistent
    grid (several tiles per workgroup) under local updates."""
    p = W.dubins_problem(31)
    V0, _, _ = hjrlib.solve(p.grid, p.dyn, p.l, None, **hjrlib.problem_options(p))
    l2 = np.minimum(p.l, W.disk_sdf(p.grid, (3.0, 3.0), 0.5))
    ref = hjrlib.solve(p.grid, p.dyn, l2, V0, **hjrlib.problem_options(p))
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    got = hjrlib.solve(p.grid, p.dyn, l2, V0, local_updates=1, **hjrlib.problem_options(p))
    _same(ref, got)


def test_batch_mixes_local_and_full_instances(gpu, hjrlib):
    p = W.dubins_problem(31)
    V0, _, _ = hjrlib.solve(p.grid, p.dyn, p.l, None, **hjrlib.problem_options(p))
    l2 = np.minimum(p.l, W.disk_sdf(p.grid, (3.0, 3.0), 0.5))
    q = W.di_box_problem(101)
    qo = dict(spatial=1, temporal=1, cfl=0.8, precision=0)
    cases = [(p, l2, V0, dict(hjrlib.problem_options(p), local_updates=1)),
             (q, q.l, None, qo),
             (q, q.l, None, dict(qo, local_updates=1)),
             (p, l2, V0, hjrlib.problem_options(p))]
    Vs, rs, sts = hjrlib.batch_solve([(c[0].grid, c[0].dyn) for c in cases], [c[1] for c in cases],
                                     [c[2] for c in cases], [c[3] for c in cases])
    for (pp, ll, kk, o), V, r, st in zip(cases, Vs, rs, sts):
        Va, ra, sa = hjrlib.solve(pp.grid, pp.dyn, ll, kk, **dict(o, local_updates=0))
        assert st == sa and np.array_equal(V, Va)
        assert (r["iterations"], r["polish_iterations"]) == (ra["iterations"], ra["polish_iterations"])


def test_serving_context_local_updates_bitwise(gpu, hjrlib):
    """Requests with local updates through the serving context, beside one without: each result
    is bitwise the full-update solve's."""
    torch = __import__("torch")
    d = W.di_box_problem(301, ubar=1.0, dbar=0.1)
    opts = dict(spatial=1, temporal=1, cfl=0.8, tol=1e-6, precision=0)
    V0, _, _ = hjrlib.solve(d.grid, d.dyn, d.l, None, **opts)
    l2 = np.minimum(d.l, W.box_sdf(d.grid, (0.6, 0.6), (0.05, 0.05)))
    p = W.dubins_problem(31)
    cases = [(d, l2, V0, dict(opts, local_updates=1)), (d, l2, V0, opts),
             (p, p.l, None, dict(hjrlib.problem_options(p), local_updates=1))]
    dev = "cuda:0"
    ls = [torch.tensor(c[1], device=dev) for c in cases]
    ks = [None if c[2] is None else torch.tensor(c[2], device=dev) for c in cases]
    outs = [torch.empty_like(l) for l in ls]
    with hjrlib.Context(0) as ctx:
        ts = [ctx.submit(c[0].grid, c[0].dyn, l, k, V, **c[3]) for c, l, k, V in zip(cases, ls, ks, outs)]
        ctx.drain()
        res = [ctx.poll(t) for t in ts]
    torch.cuda.synchronize()
    for c, V, (st, r) in zip(cases, outs, res):
        Va, ra, sa = hjrlib.solve(c[0].grid, c[0].dyn, c[1], c[2], **dict(c[3], local_updates=0))
        assert st == sa and r["iterations"] == ra["iterations"]
        assert np.array_equal(V.cpu().numpy().reshape(c[0].grid.shape), Va)
    assert res[0][1]["node_updates"] < res[1][1]["node_updates"]
