"""Seeded synthetic problem generators shared by the tests, the smoke check and the benchmark.

This module only builds inputs: grids, model parameters, target functions l and warm-start
functions k sampled at grid nodes.  It holds none of the solver's arithmetic (no derivative,
Hamiltonian, time step or projection) so that the GPU library and the FP64 oracle, which both
consume these inputs, stay independent of each other.

The problems follow the paper's examples where it gives them (the double integrator of
Sec. II-A, eq. (2), with the strip target |p| <= 2 of Sec. II-B.1) and otherwise the benchmark
problem set: a 2-D double integrator with a box obstacle, a 3-D Dubins car with a disk obstacle,
a 4-D unicycle among two disks, a 6-D quadrotor in a walled room, and a 64-instance mixed batch.
Target functions are signed distances to the unsafe set (Sec. II-B.1: l <= 0 exactly on the
unsafe set).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

SEED = 20190318

DYN_DOUBLE_INTEGRATOR = 1
DYN_DUBINS3 = 2
DYN_UNICYCLE4 = 3
DYN_QUAD6 = 4
DYN_QUAD10_XY = 5
DYN_QUAD10_Z = 6

DYN_NDIM = {DYN_DOUBLE_INTEGRATOR: 2, DYN_DUBINS3: 3, DYN_UNICYCLE4: 4, DYN_QUAD6: 6, DYN_QUAD10_XY: 4,
            DYN_QUAD10_Z: 2}
DYN_NPARAMS = {DYN_DOUBLE_INTEGRATOR: 3, DYN_DUBINS3: 4, DYN_UNICYCLE4: 4, DYN_QUAD6: 9, DYN_QUAD10_XY: 6,
               DYN_QUAD10_Z: 6}


@dataclass(frozen=True)
class Grid:
    """Uniform grid in C order (last dimension contiguous).

    Non-periodic dimension: ``n`` nodes from ``lo`` to ``hi`` inclusive.
    Periodic dimension: ``n`` nodes from ``lo``, spacing ``(hi - lo) / n``, ``hi`` excluded.
    """

    n: tuple
    lo: tuple
    hi: tuple
    periodic: tuple = ()

    def __post_init__(self):
        per = tuple(bool(p) for p in self.periodic) if self.periodic else (False,) * len(self.n)
        object.__setattr__(self, "n", tuple(int(v) for v in self.n))
        object.__setattr__(self, "lo", tuple(float(v) for v in self.lo))
        object.__setattr__(self, "hi", tuple(float(v) for v in self.hi))
        object.__setattr__(self, "periodic", per)
        if not (len(self.n) == len(self.lo) == len(self.hi) == len(self.periodic)):
            raise ValueError("grid field lengths differ")

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def shape(self) -> tuple:
        return self.n

    @property
    def size(self) -> int:
        return int(np.prod(self.n, dtype=np.int64))

    @property
    def periodic_mask(self) -> int:
        return sum(1 << i for i, p in enumerate(self.periodic) if p)

    def spacing(self, d: int) -> float:
        if self.periodic[d]:
            return (self.hi[d] - self.lo[d]) / self.n[d]
        return (self.hi[d] - self.lo[d]) / (self.n[d] - 1)

    def axis(self, d: int) -> np.ndarray:
        """Node positions along dimension d (lo + j * spacing)."""
        return self.lo[d] + np.arange(self.n[d], dtype=np.float64) * self.spacing(d)

    def mesh(self) -> list:
        """Broadcastable node-coordinate arrays, one per dimension."""
        out = []
        for d in range(self.ndim):
            shp = [1] * self.ndim
            shp[d] = self.n[d]
            out.append(self.axis(d).reshape(shp))
        return out

    def sub_box(self, dims: Sequence[int]) -> list:
        return [self.mesh()[d] for d in dims]


@dataclass(frozen=True)
class Dynamics:
    """A model id and its parameter vector (layouts documented in include/hjr.h)."""

    id: int
    params: tuple

    def __post_init__(self):
        object.__setattr__(self, "params", tuple(float(p) for p in self.params))
        if self.id not in DYN_NDIM or len(self.params) != DYN_NPARAMS[self.id]:
            raise ValueError(f"bad dynamics id/params: {self.id} {self.params}")

    @property
    def ndim(self) -> int:
        return DYN_NDIM[self.id]


def double_integrator(ubar=1.0, b=1.0, dbar=0.0) -> Dynamics:
    """x1' = x2 + d, x2' = b u, |u| <= ubar, |d| <= dbar (Sec. II-A, eq. (2))."""
    return Dynamics(DYN_DOUBLE_INTEGRATOR, (ubar, b, dbar))


def dubins3(v=1.0, ubar=1.5, dbar1=0.1, dbar2=None) -> Dynamics:
    return Dynamics(DYN_DUBINS3, (v, ubar, dbar1, dbar1 if dbar2 is None else dbar2))


def unicycle4(ubar1=1.0, ubar2=0.5, dbar=0.1, box=False) -> Dynamics:
    return Dynamics(DYN_UNICYCLE4, (ubar1, ubar2, dbar, 1.0 if box else 0.0))


def quad6(m=1.2, dbar=(0.5, 0.5, 0.5), g=9.81, phi_max=0.3, theta_max=0.3, tmin=5.0, tmax=20.0) -> Dynamics:
    return Dynamics(DYN_QUAD6, (g, m, phi_max, theta_max, tmin, tmax) + tuple(dbar))


# The 10-D near-hover quadrotor of Sec. VI (eq. (Quad10D_dyn)) with the parameters given there:
# d0 = 10, d1 = 8, n0 = 10, k_T = 4.55, |S_x|, |S_y| <= 10 degrees, 0 <= T_z <= 2g.  It splits
# into two identical horizontal 4-D subsystems and one vertical 2-D subsystem.
G = 9.81


# The scenario of Sec. VI: (mass, horizontal disturbance bound) before and after the change.
QUAD10_SCENARIOS = {"base": (5.0, 1.0), "heavier": (5.25, 1.5), "lighter": (4.8, 0.95)}

# The per-step discount factor of the discounted-reachability comparison (Sec. V, Table 1).
TABLE1_DISCOUNT = 0.999


def quad10_xy(dbar=1.0, g=G, d0=10.0, d1=8.0, n0=10.0, smax=math.radians(10.0)) -> Dynamics:
    """Horizontal subsystem (p, v, theta, omega): p' = v + d, v' = g tan(theta),
    theta' = -d1 theta + omega, omega' = -d0 theta + n0 S, |S| <= smax, |d| <= dbar."""
    return Dynamics(DYN_QUAD10_XY, (g, d0, d1, n0, smax, dbar))


def quad10_z(m=5.0, dbar=1.0, g=G, kt=4.55, tmin=0.0, tmax=2 * G) -> Dynamics:
    """Vertical subsystem (p_z, v_z): p_z' = v_z + d, v_z' = (k_T/m) T - g, T in [tmin, tmax]."""
    return Dynamics(DYN_QUAD10_Z, (g, kt, m, tmin, tmax, dbar))


# --------------------------------------------------------------------------------------------
# Target functions (signed distances sampled at the nodes, FP64)
# --------------------------------------------------------------------------------------------

def box_sdf(grid: Grid, center: Sequence[float], half: Sequence[float], dims: Optional[Sequence[int]] = None) -> np.ndarray:
    """Exact Euclidean signed distance to the axis-aligned box |x_i - c_i| <= h_i over `dims`.

    Outside: norm of the per-axis excess; inside: the largest (negative) per-axis margin."""
    dims = list(range(len(center))) if dims is None else list(dims)
    mesh = grid.mesh()
    q = [np.abs(mesh[d] - c) - h for d, c, h in zip(dims, center, half)]
    outside = np.sqrt(sum(np.maximum(qi, 0.0) ** 2 for qi in q))
    inside = q[0]
    for qi in q[1:]:
        inside = np.maximum(inside, qi)
    out = outside + np.minimum(inside, 0.0)
    return np.ascontiguousarray(np.broadcast_to(out, grid.shape), dtype=np.float64)


def disk_sdf(grid: Grid, center: Sequence[float], radius: float, dims=(0, 1)) -> np.ndarray:
    mesh = grid.mesh()
    r = np.sqrt((mesh[dims[0]] - center[0]) ** 2 + (mesh[dims[1]] - center[1]) ** 2) - radius
    return np.ascontiguousarray(np.broadcast_to(r, grid.shape), dtype=np.float64)


def disks_sdf(grid: Grid, centers, radii, dims=(0, 1)) -> np.ndarray:
    out = None
    for c, r in zip(centers, radii):
        s = disk_sdf(grid, c, r, dims)
        out = s if out is None else np.minimum(out, s)
    return out


def strip_target(grid: Grid, half_width=2.0, dim=0) -> np.ndarray:
    """The running example's unsafe strip |p| <= 2 (Sec. II-B.1): l = |p| - 2."""
    mesh = grid.mesh()
    out = np.abs(mesh[dim]) - half_width
    return np.ascontiguousarray(np.broadcast_to(out, grid.shape), dtype=np.float64)


def room_target(grid: Grid, half_room=4.0, dims=(0, 1, 2)) -> np.ndarray:
    """Walls of a cube room are unsafe: l = min_i (half_room - |p_i|)."""
    mesh = grid.mesh()
    out = None
    for d in dims:
        s = half_room - np.abs(mesh[d])
        out = s if out is None else np.minimum(out, s)
    return np.ascontiguousarray(np.broadcast_to(out, grid.shape), dtype=np.float64)


# --------------------------------------------------------------------------------------------
# Problem records
# --------------------------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    grid: Grid
    dyn: Dynamics
    l: np.ndarray
    spatial: int = 1          # 1 upwind, 5 WENO5
    temporal: int = 1         # 1 Euler, 3 TVD-RK3
    cfl: float = 0.8
    tol: float = 1e-6
    game: int = 0             # 0 avoid, 1 reach
    meta: dict = field(default_factory=dict)


def di_box_problem(n=101, ubar=1.0, dbar=0.0, b=1.0, half=0.2) -> Problem:
    """2-D double integrator on [-1,1]^2, box obstacle |x_i| <= 0.2, upwind + Euler, CFL 0.8."""
    g = Grid((n, n), (-1.0, -1.0), (1.0, 1.0))
    return Problem(f"di{n}", g, double_integrator(ubar, b, dbar), box_sdf(g, (0.0, 0.0), (half, half)),
                   spatial=1, temporal=1, cfl=0.8, tol=1e-6)


def di_strip_problem(n=81, ubar=1.0, b=1.0, dbar=0.0, extent=5.0, spatial=1, temporal=1, cfl=0.8) -> Problem:
    """The running example: strip target |p| <= 2 on [-extent, extent]^2 (Sec. II-A/B)."""
    g = Grid((n, n), (-extent, -extent), (extent, extent))
    return Problem(f"distrip{n}", g, double_integrator(ubar, b, dbar), strip_target(g),
                   spatial=spatial, temporal=temporal, cfl=cfl)


def dubins_problem(n=101, ntheta=None, ubar=1.5, dbar=0.1, v=1.0, radius=1.0, center=(0.0, 0.0), cfl=0.5,
                   scheme="weno") -> Problem:
    """3-D Dubins car on [-5,5]^2 x [-pi,pi) (theta periodic), disk obstacle.  scheme "weno":
    WENO5 + TVD-RK3 at CFL `cfl`; "upwind": first-order upwind + forward Euler at CFL 0.8."""
    nt = n if ntheta is None else ntheta
    g = Grid((n, n, nt), (-5.0, -5.0, -math.pi), (5.0, 5.0, math.pi), (False, False, True))
    sp, tp, c = (5, 3, cfl) if scheme == "weno" else (1, 1, 0.8)
    return Problem(f"dubins{n}", g, dubins3(v, ubar, dbar), disk_sdf(g, center, radius),
                   spatial=sp, temporal=tp, cfl=c)


def unicycle_centers(seed=SEED):
    rng = np.random.default_rng(seed)
    centers = rng.uniform(-4.0, 4.0, size=(2, 2))
    radii = rng.uniform(0.5, 1.5, size=2)
    ang = rng.uniform(0.0, 2 * math.pi)
    moved = centers.copy()
    moved[0] += 0.3 * np.array([math.cos(ang), math.sin(ang)])
    return centers, radii, moved


def unicycle_problem(n=61, moved=False, seed=SEED, cfl=0.5) -> Problem:
    """4-D unicycle on [-5,5]^2 x [-pi,pi) x [0,2], two seeded disks (radius 0.5-1.5)."""
    g = Grid((n, n, n, n), (-5.0, -5.0, -math.pi, 0.0), (5.0, 5.0, math.pi, 2.0), (False, False, True, False))
    centers, radii, mv = unicycle_centers(seed)
    l = disks_sdf(g, mv if moved else centers, radii)
    return Problem(f"unicycle{n}", g, unicycle4(1.0, 0.5, 0.1), l, spatial=5, temporal=3, cfl=cfl,
                   meta={"centers": (mv if moved else centers).tolist(), "radii": radii.tolist()})


def quad6_problem(n=25, m=1.2, dbar=(0.5, 0.5, 0.5), cfl=0.8, target="obstacle") -> Problem:
    """6-D quadrotor translation, v in [-3,3]^3.

    target "obstacle" (default): a cube obstacle |p_i| <= 1 in p in [-5,5]^3, l = its exact
    signed distance; far from it V = l, so the iteration settles.  target "room": p in [-6,6]^3
    with the walls |p_i| >= 4 unsafe, l = min_i (4 - |p_i|); l is unbounded below outside the
    room and the linearly extrapolated edges let V drift down there, so that variant does not
    settle and is kept for fixed-step checks only.  Scheme: upwind + Euler (monotone)."""
    if target == "room":
        g = Grid((n,) * 6, (-6.0, -6.0, -6.0, -3.0, -3.0, -3.0), (6.0, 6.0, 6.0, 3.0, 3.0, 3.0))
        l = room_target(g)
    else:
        g = Grid((n,) * 6, (-5.0, -5.0, -5.0, -3.0, -3.0, -3.0), (5.0, 5.0, 5.0, 3.0, 3.0, 3.0))
        l = box_sdf(g, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), dims=(0, 1, 2))
    return Problem(f"quad{n}", g, quad6(m=m, dbar=dbar), l, spatial=1, temporal=1, cfl=cfl)


def quad10_problems(m=5.0, dbar_xy=1.0, dbar_z=1.0, n_xy=31, n_z=101, scheme="upwind") -> list:
    """The three subsystems of the 10-D near-hover quadrotor (Sec. VI) as avoid problems: x and y
    (identical) with a wall slab |p| <= 1 to stay out of, on p in [-6,6], v in [-4,4],
    theta in [-0.4,0.4], omega in [-4,4]; z with the floor p_z <= 0 to stay above, on
    p_z in [-2,8], v_z in [-6,6].  Targets and grids are readings (the paper gives neither).
    scheme "upwind": first-order upwind + forward Euler at CFL 0.8; "weno": WENO5 + TVD-RK3 at 0.5."""
    sp, tp, cfl = (1, 1, 0.8) if scheme == "upwind" else (5, 3, 0.5)
    gxy = Grid((n_xy,) * 4, (-6.0, -4.0, -0.4, -4.0), (6.0, 4.0, 0.4, 4.0))
    lxy = np.broadcast_to(np.abs(gxy.mesh()[0]) - 1.0, gxy.shape).copy()
    gz = Grid((n_z, n_z), (-2.0, -6.0), (8.0, 6.0))
    lz = np.broadcast_to(gz.mesh()[0], gz.shape).copy()
    out = []
    for axis in ("x", "y"):
        out.append(Problem(f"quad10-{axis}{n_xy}", gxy, quad10_xy(dbar_xy), lxy, spatial=sp, temporal=tp, cfl=cfl))
    out.append(Problem(f"quad10-z{n_z}", gz, quad10_z(m, dbar_z), lz, spatial=sp, temporal=tp, cfl=cfl))
    return out


def batch_problems(count=64, seed=SEED, n2=(51, 201), n3=(41, 121)) -> list:
    """Mixed batch: 50/50 double integrator (2-D) / Dubins (3-D), side length uniform in range,
    control bound U[0.5, 2], disturbance bound U[0, 0.2], obstacle centre uniform in the domain.
    Every instance uses first-order upwind + forward Euler at CFL 0.8: the monotone scheme has a
    steady state on each of them, while WENO5 + TVD-RK3 has none on 20 of the 32 Dubins
    instances (with an obstacle off the origin its iterates keep circulating; the FP64 oracle
    shows the same) and on the double integrator's box corners."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        is3 = bool(rng.integers(0, 2))
        ubar = float(rng.uniform(0.5, 2.0))
        dbar = float(rng.uniform(0.0, 0.2))
        if is3:
            n = int(rng.integers(n3[0], n3[1] + 1))
            c = rng.uniform(-5.0, 5.0, size=2)
            g = Grid((n, n, n), (-5.0, -5.0, -math.pi), (5.0, 5.0, math.pi), (False, False, True))
            p = Problem(f"b{i}-dubins{n}", g, dubins3(1.0, ubar, dbar), disk_sdf(g, c, 1.0),
                        spatial=1, temporal=1, cfl=0.8)
        else:
            n = int(rng.integers(n2[0], n2[1] + 1))
            c = rng.uniform(-1.0, 1.0, size=2)
            g = Grid((n, n), (-1.0, -1.0), (1.0, 1.0))
            p = Problem(f"b{i}-di{n}", g, double_integrator(ubar, 1.0, dbar), box_sdf(g, c, (0.2, 0.2)),
                        spatial=1, temporal=1, cfl=0.8)
        out.append(p)
    return out


def random_circles_k(grid: Grid, count=12, seed=SEED, dims=(0, 1)) -> np.ndarray:
    """Warm-start function whose zero sublevel set is the complement of random circles
    (the experiment of Sec. IV-D): k = -(signed distance to the union of circles)."""
    rng = np.random.default_rng(seed)
    lo = [grid.lo[d] for d in dims]
    hi = [grid.hi[d] for d in dims]
    centers = [rng.uniform(lo, hi) for _ in range(count)]
    span = min(h - l_ for l_, h in zip(lo, hi))
    radii = rng.uniform(0.05 * span, 0.15 * span, size=count)
    return -disks_sdf(grid, centers, radii, dims)


def smooth_field(grid: Grid, seed=SEED, kinks=True) -> np.ndarray:
    """A random smooth field (plus optional kinks) for single-operator parity checks."""
    rng = np.random.default_rng(seed)
    mesh = grid.mesh()
    out = np.zeros(grid.shape)
    for _ in range(4):
        w = rng.normal(size=grid.ndim)
        ph = rng.uniform(0, 2 * math.pi)
        arg = ph
        for d in range(grid.ndim):
            span = grid.hi[d] - grid.lo[d]
            arg = arg + w[d] * 2 * math.pi / span * mesh[d]
        out = out + rng.uniform(0.2, 1.0) * np.sin(arg)
    if kinks:
        c = [rng.uniform(grid.lo[d], grid.hi[d]) for d in range(grid.ndim)]
        r = np.sqrt(sum((mesh[d] - c[d]) ** 2 for d in range(grid.ndim)))
        out = np.minimum(out, r - 0.3 * (grid.hi[0] - grid.lo[0]) / 2)
    return np.ascontiguousarray(out, dtype=np.float64)
