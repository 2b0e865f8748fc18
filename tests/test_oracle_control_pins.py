"""Pins of the oracle's safe-control query (Sec. II-B.2, eq. (uOpt)) to facts that do not come from
the oracle itself: exact gradients of linear and quadratic value functions (the one-sided
derivative averages and multilinear interpolation reproduce them), second-order accuracy on a
smooth periodic function, and the optimal control checked against a dense lattice search of
argmax_u min_d <p, f(x, u, d)> with the model equations written out here.
"""
import math

import numpy as np
import pytest

from paper_1903_07715_amd import workloads as W
from test_oracle_pins import _flow_np, _lattices

AVOID, REACH = 0, 1


def _rand_states(grid, rng, count, margin=0.0):
    lo = np.array(grid.lo) + margin * np.array([grid.spacing(d) for d in range(grid.ndim)])
    hi = np.array(grid.hi) - margin * np.array([grid.spacing(d) for d in range(grid.ndim)])
    return rng.uniform(lo, hi, size=(count, grid.ndim))


@pytest.mark.parametrize("ndim", [2, 3, 4])
def test_linear_value_gives_exact_gradient_everywhere(orc, ndim):
    """V = a.x + b: every one-sided difference equals a_i, also at the edges (linear ghost
    extrapolation continues a linear function), and interpolation of a constant gradient and of
    a linear V is exact; states outside the box are clamped onto it."""
    rng = np.random.default_rng(11 + ndim)
    n = (9, 11, 7, 8)[:ndim]
    g = W.Grid(n, tuple(-1.0 - 0.5 * d for d in range(ndim)), tuple(1.0 + 0.25 * d for d in range(ndim)))
    a = rng.normal(size=ndim)
    b = 0.3
    V = b + sum(a[d] * m for d, m in enumerate(g.mesh()))
    dyn = {2: W.double_integrator(1.0, 1.0, 0.1), 3: W.dubins3(1.0, 1.0, 0.1, 0.1),
           4: W.unicycle4(1.0, 0.5, 0.1)}[ndim]
    x = _rand_states(g, rng, 200)
    x[:20] *= 3.0  # outside the box
    for spatial in (orc.UPWIND1, orc.WENO5):
        u, p, v = orc.safe_control(g, dyn, V, x, spatial=spatial)
        assert np.abs(p - a).max() < 1e-11
        xc = np.clip(x, g.lo, g.hi)
        assert np.abs(v - (b + xc @ a)).max() < 1e-11


def test_quadratic_value_gives_exact_gradient_inside(orc):
    """V = x'Qx + c.x: the average of the one-sided differences is the central difference (upwind)
    or a convex combination of exact quadratic interpolants (WENO5), exact for quadratics away
    from the edges; the gradient 2Qx + c is affine in each coordinate separately, which
    multilinear interpolation reproduces exactly."""
    rng = np.random.default_rng(5)
    g = W.Grid((15, 13, 17), (-2.0, -1.0, -1.5), (2.0, 1.5, 1.0))
    Q = rng.normal(size=(3, 3))
    Q = Q + Q.T
    c = rng.normal(size=3)
    M = g.mesh()
    V = sum(Q[i, j] * M[i] * M[j] for i in range(3) for j in range(3)) + sum(c[i] * M[i] for i in range(3))
    x = _rand_states(g, rng, 300, margin=3.0)
    for spatial in (orc.UPWIND1, orc.WENO5):
        _, p, _ = orc.safe_control(g, W.dubins3(1.0, 1.0, 0.0, 0.0), V, x, spatial=spatial)
        exact = 2 * x @ Q + c
        assert np.abs(p - exact).max() < 1e-9 * (1 + np.abs(exact).max())


def test_periodic_gradient_is_second_order(orc):
    """V = sin(theta) + 0.5 x on a grid periodic in theta: the interpolated d/dtheta matches
    cos(theta) with an error that falls about 4x when the spacing halves, including states whose
    cell wraps around the period and states given outside one period."""
    rng = np.random.default_rng(3)
    errs = []
    for n in (32, 64):
        g = W.Grid((5, 5, n), (-1.0, -1.0, -math.pi), (1.0, 1.0, math.pi), (False, False, True))
        M = g.mesh()
        V = np.broadcast_to(np.sin(M[2]) + 0.5 * M[0], g.shape).copy()
        x = _rand_states(g, rng, 400)
        x[:50, 2] = rng.uniform(math.pi - 0.05, math.pi, size=50)  # last cell: wraps to node 0
        x[50:100, 2] += 2 * math.pi * rng.integers(-3, 4, size=50)
        _, p, _ = orc.safe_control(g, W.dubins3(1.0, 1.0, 0.0, 0.0), V, x, spatial=orc.UPWIND1)
        assert np.abs(p[:, 0] - 0.5).max() < 1e-12
        errs.append(np.abs(p[:, 2] - np.cos(x[:, 2])).max())
    assert errs[0] < 0.5 * (2 * math.pi / 32) ** 2
    assert 3.0 < errs[0] / errs[1] < 5.0


@pytest.mark.parametrize("dyn", [W.double_integrator(1.0, 0.8, 0.3), W.double_integrator(1.0, -0.6, 0.1),
                                 W.dubins3(1.0, 1.5, 0.1, 0.2), W.unicycle4(1.0, 0.5, 0.1),
                                 W.unicycle4(1.0, 0.5, 0.1, box=True), W.quad6(1.2, (0.5, 0.3, 0.4)),
                                 W.quad10_xy(1.2), W.quad10_z(5.25, 0.7)])
@pytest.mark.parametrize("game", [AVOID, REACH])
def test_optimal_control_attains_lattice_optimum(orc, dyn, game):
    """u* attains max_u min_d <p, f> (avoid) or min_u max_d (reach) over dense lattices of the
    control and disturbance sets, and lies in the control set."""
    rng = np.random.default_rng(17)
    Ug, Dg = _lattices(dyn, k=9)
    q = dyn.params
    for _ in range(8):
        x = rng.uniform(-2, 2, size=dyn.ndim)
        if dyn.id == W.DYN_UNICYCLE4:
            x[3] = rng.uniform(0, 2)
        if dyn.id == W.DYN_QUAD10_XY:
            x[2] = rng.uniform(-0.4, 0.4)
        p = rng.normal(size=dyn.ndim)

        def inner(u):
            f = _flow_np(dyn, x, u, Dg.T)
            s = sum(pi * np.asarray(fi) for pi, fi in zip(p, f))
            return np.min(s) if game == AVOID else np.max(s)

        u = orc.optimal_control(dyn, x, p, game)
        lattice = np.array([inner(uu) for uu in Ug])
        best = lattice.max() if game == AVOID else lattice.min()
        got = inner(u)
        tol = 1e-12 * (1 + abs(best))
        assert (got >= best - tol) if game == AVOID else (got <= best + tol)
        if dyn.id == W.DYN_QUAD6:
            assert abs(u[0]) <= q[3] + 1e-15 and abs(u[1]) <= q[2] + 1e-15 and q[4] <= u[2] <= q[5]
        elif dyn.id == W.DYN_UNICYCLE4:
            assert abs(u[0]) <= q[0] + 1e-15 and abs(u[1]) <= q[1] + 1e-15
        elif dyn.id == W.DYN_QUAD10_XY:
            assert abs(u[0]) <= q[4] + 1e-15
        elif dyn.id == W.DYN_QUAD10_Z:
            assert q[3] <= u[0] <= q[4]
        else:
            assert abs(u[0]) <= (q[0] if dyn.id == W.DYN_DOUBLE_INTEGRATOR else q[1]) + 1e-15


def test_zero_gradient_component_picks_upper_bound(orc):
    """A control whose coefficient in <p, f> vanishes is optimal at any value; the rule picks its
    upper bound (documented tie rule), the other controls still follow their gradient."""
    uni = W.unicycle4(1.0, 0.5, 0.1)
    x = np.array([0.1, 0.2, 0.3, 1.0])
    u = orc.optimal_control(uni, x, np.array([0.3, -0.2, 0.0, -1.0]), AVOID)
    assert u[0] == 1.0 and u[1] == -0.5
    u = orc.optimal_control(uni, x, np.array([0.3, -0.2, 2.0, 0.0]), REACH)
    assert u[0] == -1.0 and u[1] == 0.5
    quad = W.quad6(1.2, (0.5, 0.3, 0.4))
    q = quad.params
    u = orc.optimal_control(quad, np.zeros(6), np.zeros(6), AVOID)
    assert list(u) == [q[3], q[2], q[5]]


def test_safe_control_brakes_toward_the_obstacle(orc):
    """Running example (Sec. II-A/B): on the double integrator's converged avoid value function,
    a state right of the unsafe strip moving toward it gets full braking (u = +ubar), and the
    mirrored state left of the strip, also moving toward it, gets full braking the other way."""
    pr = W.di_strip_problem(61, spatial=orc.UPWIND1, temporal=orc.EULER, cfl=0.8)
    V, info = orc.solve(pr.grid, pr.dyn, pr.l, max_iter=20000, **orc.problem_opts(pr))
    assert info["converged"] == 1
    x = np.array([[3.0, -1.5], [-3.0, 1.5]])
    u, p, v = orc.safe_control(pr.grid, pr.dyn, V, x)
    ubar, b = pr.dyn.params[0], pr.dyn.params[1]
    assert u[0, 0] == ubar * np.sign(b) and u[1, 0] == -ubar * np.sign(b)
