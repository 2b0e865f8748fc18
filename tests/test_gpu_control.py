"""GPU parity of the safe-control query (Sec. II-B.2, eq. (uOpt)) with the oracle, through the C ABI.

The nodal gradient is compared at every node of small grids of every dimension, periodic dims
and both schemes included; the query outputs p and v at random states (inside, outside the box,
on nodes, across the periodic seam, non-finite) to FP64 rounding; the control u exactly wherever
the deciding coefficient is clear of rounding, and otherwise only for lying on one of the two
bounds (both are optimal up to rounding there).
"""
import math

import numpy as np
import pytest

from paper_1903_07715_amd import workloads as W

pytestmark = pytest.mark.gpu

AVOID, REACH = 0, 1


def _cases():
    return [
        ("di", W.Grid((31, 27), (-1.0, -1.5), (1.0, 1.5)), W.double_integrator(0.8, -1.3, 0.1)),
        ("dubins", W.Grid((17, 19, 21), (-5.0, -5.0, -math.pi), (5.0, 5.0, math.pi), (False, False, True)),
         W.dubins3(1.0, 1.5, 0.1, 0.05)),
        ("unicycle", W.Grid((9, 8, 11, 7), (-5.0, -5.0, -math.pi, 0.0), (5.0, 5.0, math.pi, 2.0),
                            (False, False, True, False)), W.unicycle4(1.0, 0.5, 0.1)),
        ("quad", W.Grid((7, 7, 8, 7, 7, 9), (-5.0, -5.0, -5.0, -3.0, -3.0, -3.0), (5.0, 5.0, 5.0, 3.0, 3.0, 3.0)),
         W.quad6(1.2, (0.5, 0.3, 0.4))),
        ("quad10-xy", W.Grid((9, 8, 11, 7), (-6.0, -4.0, -0.4, -4.0), (6.0, 4.0, 0.4, 4.0)), W.quad10_xy(1.2)),
        ("quad10-z", W.Grid((37, 31), (-2.0, -6.0), (8.0, 6.0)), W.quad10_z(5.25, 0.7)),
    ]


def _coef(dyn, p):
    """The coefficient of each control in <p, f> (its sign decides the control)."""
    q = dyn.params
    if dyn.id == W.DYN_DOUBLE_INTEGRATOR:
        return np.stack([q[1] * p[:, 1]], 1)
    if dyn.id == W.DYN_DUBINS3:
        return p[:, 2:3]
    if dyn.id == W.DYN_UNICYCLE4:
        return p[:, 2:4]
    if dyn.id == W.DYN_QUAD10_XY:
        return q[3] * p[:, 3:4]
    if dyn.id == W.DYN_QUAD10_Z:
        return q[1] / q[2] * p[:, 1:2]
    return np.stack([q[0] * p[:, 3], -q[0] * p[:, 4], p[:, 5]], 1)


def _bounds(dyn):
    q = dyn.params
    if dyn.id == W.DYN_DOUBLE_INTEGRATOR:
        return [(-q[0], q[0])]
    if dyn.id == W.DYN_DUBINS3:
        return [(-q[1], q[1])]
    if dyn.id == W.DYN_UNICYCLE4:
        return [(-q[0], q[0]), (-q[1], q[1])]
    if dyn.id == W.DYN_QUAD10_XY:
        return [(-q[4], q[4])]
    if dyn.id == W.DYN_QUAD10_Z:
        return [(q[3], q[4])]
    return [(-q[3], q[3]), (-q[2], q[2]), (q[4], q[5])]


def _queries(grid, rng, count):
    lo, hi = np.array(grid.lo), np.array(grid.hi)
    x = rng.uniform(lo, hi, size=(count, grid.ndim))
    span = hi - lo
    x[: count // 10] = rng.uniform(lo - 0.3 * span, hi + 0.3 * span, size=(count // 10, grid.ndim))  # outside
    k = count // 10
    for i in range(k, 2 * k):  # exactly on nodes
        for d in range(grid.ndim):
            x[i, d] = grid.axis(d)[rng.integers(0, grid.n[d])]
    for d in range(grid.ndim):
        if grid.periodic[d]:
            x[2 * k: 3 * k, d] = hi[d] - rng.uniform(0, 0.5 * grid.spacing(d), size=k)  # last cell, wraps
            x[3 * k: 4 * k, d] += span[d] * rng.integers(-2, 3, size=k)                  # other periods
    x[-3] = np.nan
    x[-2, 0] = np.inf
    return x


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


@pytest.mark.parametrize("spatial", [1, 5])
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_gradient_matches_oracle_at_every_node(gpu, hjrlib, orc, case, spatial):
    torch = __import__("torch")
    name, g, dyn = case
    V = W.smooth_field(g, seed=3)
    Vt = _dev(torch, V)
    gt = torch.empty((g.ndim + 1) * g.size, dtype=torch.float64, device="cuda:0")
    print(f"[control] gradient {name} spatial={spatial} nodes={g.size}", flush=True)
    hjrlib.gradient_device(g, Vt, gt, spatial=spatial)
    torch.cuda.synchronize()
    table = gt.cpu().numpy().reshape(g.size, g.ndim + 1)
    ref = orc.gradient_at(g, V, np.arange(g.size), spatial=spatial)
    scale = 1.0 + np.abs(ref).max()
    assert np.abs(table[:, :g.ndim] - ref).max() <= 1e-12 * scale
    assert np.array_equal(table[:, g.ndim], V.ravel())


@pytest.mark.parametrize("game", [AVOID, REACH])
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_safe_control_matches_oracle(gpu, hjrlib, orc, case, game):
    torch = __import__("torch")
    name, g, dyn = case
    rng = np.random.default_rng(21)
    V = W.smooth_field(g, seed=5)
    x = _queries(g, rng, 2000)
    Vt, xt = _dev(torch, V), _dev(torch, x)
    gt = torch.empty((g.ndim + 1) * g.size, dtype=torch.float64, device="cuda:0")
    nu = hjrlib.num_controls(dyn)
    ut = torch.empty(x.shape[0] * nu, dtype=torch.float64, device="cuda:0")
    pt = torch.empty(x.shape[0] * g.ndim, dtype=torch.float64, device="cuda:0")
    vt = torch.empty(x.shape[0], dtype=torch.float64, device="cuda:0")
    print(f"[control] query {name} game={game} queries={x.shape[0]}", flush=True)
    hjrlib.gradient_device(g, Vt, gt, spatial=1)
    hjrlib.safe_control_device(g, dyn, gt, xt, ut, p=pt, v=vt, game=game)
    torch.cuda.synchronize()
    u = ut.cpu().numpy().reshape(-1, nu)
    p = pt.cpu().numpy().reshape(-1, g.ndim)
    v = vt.cpu().numpy()
    uo, po, vo = orc.safe_control(g, dyn, V, x, game=game, spatial=1)
    bad = ~np.isfinite(x).all(axis=1)
    assert np.isnan(u[bad]).all() and np.isnan(p[bad]).all() and np.isnan(v[bad]).all()
    assert np.isnan(uo[bad]).all()
    ok = ~bad
    scale = 1.0 + np.abs(po[ok]).max()
    assert np.abs(p[ok] - po[ok]).max() <= 1e-12 * scale
    assert np.abs(v[ok] - vo[ok]).max() <= 1e-12 * (1.0 + np.abs(vo[ok]).max())
    coef = _coef(dyn, po[ok])
    clear = np.abs(coef) > 1e-9 * scale * (1.0 + np.abs(np.asarray(dyn.params)).max())
    assert np.array_equal(u[ok][clear], uo[ok][clear])
    for i, (lo, hi) in enumerate(_bounds(dyn)):
        assert np.isin(u[ok][:, i], [lo, hi]).all()
    assert clear.mean() > 0.5


def test_safe_control_options_and_empty_batch(gpu, hjrlib, orc):
    torch = __import__("torch")
    name, g, dyn = _cases()[1]
    V = W.smooth_field(g, seed=9)
    x = _queries(g, np.random.default_rng(4), 300)[:-3]
    Vt, xt = _dev(torch, V), _dev(torch, x)
    gt = torch.empty((g.ndim + 1) * g.size, dtype=torch.float64, device="cuda:0")
    hjrlib.gradient_device(g, Vt, gt, spatial=5)
    u1 = torch.empty(x.shape[0], dtype=torch.float64, device="cuda:0")
    hjrlib.safe_control_device(g, dyn, gt, xt, u1)  # no p, no v
    u2 = torch.empty_like(u1)
    pt = torch.empty(x.shape[0] * 3, dtype=torch.float64, device="cuda:0")
    hjrlib.safe_control_device(g, dyn, gt, xt, u2, p=pt)
    empty = torch.empty(0, dtype=torch.float64, device="cuda:0")
    hjrlib.safe_control_device(g, dyn, gt, empty.reshape(0, 3), empty)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
    uo, po, _ = orc.safe_control(g, dyn, V, x, spatial=5)
    assert np.abs(pt.cpu().numpy().reshape(-1, 3) - po).max() <= 1e-12 * (1 + np.abs(po).max())


def test_safe_control_on_converged_dubins_value(gpu, hjrlib, orc):
    """The query on the benchmark problem's converged value function (101^3 Dubins car,
    WENO5 gradient), 200 000 states, checked against the oracle on a sample of them."""
    torch = __import__("torch")
    p = W.dubins_problem(101)
    g = p.grid
    lt = _dev(torch, p.l)
    Vt = torch.empty_like(lt)
    res, st = hjrlib.solve_device(g, p.dyn, lt, None, Vt, **hjrlib.problem_options(p))
    assert st == hjrlib.OK
    rng = np.random.default_rng(8)
    x = rng.uniform(g.lo, g.hi, size=(200000, 3))
    xt = _dev(torch, x)
    gt = torch.empty(4 * g.size, dtype=torch.float64, device="cuda:0")
    ut = torch.empty(x.shape[0], dtype=torch.float64, device="cuda:0")
    pt = torch.empty(3 * x.shape[0], dtype=torch.float64, device="cuda:0")
    hjrlib.gradient_device(g, Vt, gt, spatial=5)
    hjrlib.safe_control_device(g, p.dyn, gt, xt, ut, p=pt)
    torch.cuda.synchronize()
    V = Vt.cpu().numpy().reshape(g.shape)
    idx = rng.choice(x.shape[0], 3000, replace=False)
    uo, po, _ = orc.safe_control(g, p.dyn, V, x[idx], spatial=5)
    pg = pt.cpu().numpy().reshape(-1, 3)[idx]
    assert np.abs(pg - po).max() <= 1e-12 * (1 + np.abs(po).max())
    ug = ut.cpu().numpy()[idx]
    clear = np.abs(po[:, 2]) > 1e-9 * (1 + np.abs(po).max())
    assert np.array_equal(ug[clear], uo[clear, 0])
