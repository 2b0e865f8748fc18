"""The plane-march stage kernels (one thread per column walking the dim-0 planes; first-order
upwind, and WENO5 with each dim-0 interface computed once) against the flat-tile kernel and the
FP64 oracle.

The march kernels evaluate the same per-node arithmetic as the flat-tile kernels, only with the
column's offsets, edge rule and model coordinates set up once per column and the dim-0
neighbours (upwind) or dim-0 differences and interfaces (WENO5) carried in registers, so every
output and every max-change reduction must be bitwise identical to the flat kernel's, for every
scheme, model, game, precision, integrator stage, ragged grid, periodic dimension (dim 0
included) and run length (whole lines, and runs of 8, 4 and 2 planes, whose ends fall at
different distances from the grid's edges).  Configuration -16, the brick variant (pairs of rows
of dims 1..3 sharing their far neighbours through LDS), serves the 6-D upwind cases; elsewhere
the library runs the whole-line march kernel for it.  The oracle then pins the common result (FP64:
1e-12, FP32: 2e-5 of the field's scale, as in the stage parity tests).
"""
import math

import numpy as np
import pytest

from paper_1903_07715_amd import workloads as W

pytestmark = pytest.mark.gpu
SEED = W.SEED


def _cases():
    # every grid has at least 8192 columns (nodes per dim-0 plane), the march kernel's minimum
    quad = W.Grid((7, 9, 11, 13, 8, 10), (-5, -5, -5, -3, -3, -3), (5, 5, 5, 3, 3, 3))
    # periodic dims 1 and 3 (even lengths) and an odd non-periodic dim 2 between them; rows of
    # 9 x 31 = 279 columns, so the brick kernel's segments are 128, 128 and 23 columns long
    quadper = W.Grid((7, 8, 7, 8, 9, 31), (-5, -5, -5, -3, -3, -3), (5, 5, 5, 3, 3, 3),
                     (False, True, False, True, False, False))
    q10xy = W.Grid((13, 41, 23, 17), (-6.0, -4.0, -0.4, -4.0), (6.0, 4.0, 0.4, 4.0))
    uni = W.Grid((9, 31, 24, 15), (-5.0, -5.0, -math.pi, 0.0), (5.0, 5.0, math.pi, 2.0), (False, False, True, False))
    dub = W.Grid((21, 97, 101), (-5.0, -5.0, -math.pi), (5.0, 5.0, math.pi), (False, False, True))
    diper = W.Grid((37, 9001), (-1.0, -1.0), (1.0, 1.0), (True, True))  # dim 0 periodic
    q10z = W.Grid((11, 8193), (-2.0, -6.0), (8.0, 6.0))
    return [
        ("quad6", quad, W.quad6(1.2, (0.5, 0.3, 0.4))),
        ("quad6-periodic", quadper, W.quad6(1.2, (0.5, 0.3, 0.4))),
        ("quad10-xy", q10xy, W.quad10_xy(1.2)),
        ("unicycle", uni, W.unicycle4(1.0, 0.5, 0.1)),
        ("dubins", dub, W.dubins3(1.0, 1.5, 0.1, 0.05)),
        ("di-periodic", diper, W.double_integrator(1.0, 0.8, 0.3)),
        ("quad10-z", q10z, W.quad10_z(5.25, 0.7)),
    ]


def _run_stage(hjrlib, monkeypatch, cfg, g, d, stage, dt, src, vn, l, temporal, prec, game, spatial):
    import torch

    monkeypatch.setenv("HJR_NPT", cfg)
    out = torch.empty_like(vn)
    delta = hjrlib.stage_device(g, d, stage, dt, src, vn, l, out, game=game, spatial=spatial,
                                temporal=temporal, precision=prec)
    torch.cuda.synchronize()
    return out, delta


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("temporal", [1, 3], ids=["euler", "rk3"])
@pytest.mark.parametrize("game", [0, 1], ids=["avoid", "reach"])
@pytest.mark.parametrize("spatial", [1, 5], ids=["upwind", "weno5"])
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_march_stage_bitwise_equals_flat_and_matches_oracle(gpu, hjrlib, orc, monkeypatch, case, spatial, temporal,
                                                            precision, game):
    import torch

    name, g, d = case
    print(f"[march] {name} {g.n} spatial={spatial} temporal={temporal} {precision} game={game}", flush=True)
    rng = np.random.default_rng(SEED)
    Vn = W.smooth_field(g, seed=SEED)
    Vs = Vn + 0.05 * W.smooth_field(g, seed=SEED + 1, kinks=False)
    l = Vn + rng.uniform(-0.05, 0.2, size=g.shape)
    tdt = torch.float32 if precision == "fp32" else torch.float64
    prec = hjrlib.FP32 if precision == "fp32" else hjrlib.FP64
    if precision == "fp32":
        Vn, Vs, l = (a.astype(np.float32).astype(np.float64) for a in (Vn, Vs, l))
    dt = orc.cfl_dt(g, d, 0.8)
    t_vn = torch.tensor(Vn, dtype=tdt, device=gpu)
    t_vs = torch.tensor(Vs, dtype=tdt, device=gpu)
    t_l = torch.tensor(l, dtype=tdt, device=gpu)
    nodes = np.unique(np.concatenate([np.arange(0, g.size, max(1, g.size // 4000)), [g.size - 1]]))
    scale = 1.0 + np.abs(Vn).max()
    tol = 2e-5 * scale if precision == "fp32" else 1e-12 * scale
    for stage in range(1, (3 if temporal == 3 else 1) + 1):
        src = t_vn if stage == 1 else t_vs
        flat, dflat = _run_stage(hjrlib, monkeypatch, "4", g, d, stage, dt, src, t_vn, t_l, temporal, prec, game,
                                 spatial)
        for cfg in ("-1", "-8", "-4", "-2", "-16"):
            got, dgot = _run_stage(hjrlib, monkeypatch, cfg, g, d, stage, dt, src, t_vn, t_l, temporal, prec, game,
                                   spatial)
            assert torch.equal(got, flat), (name, stage, cfg, float((got.double() - flat.double()).abs().max()))
            assert (dgot is None and dflat is None) or dgot == dflat
        ref = orc.stage_at(g, d, stage, dt, (Vn if stage == 1 else Vs), Vn, l, nodes, spatial=spatial,
                           temporal=temporal, game=game)
        err = np.abs(flat.double().cpu().numpy().ravel()[nodes] - ref).max()
        assert err <= tol, (name, stage, err)


def test_march_solves_bitwise_equal_flat(gpu, hjrlib, monkeypatch):
    """Whole FP32 + FP64-polish solves of a 6-D quadrotor (13^6 = 4.8 M nodes), cold and warm:
    the march configurations and the flat one give the same iterations and bitwise the same V."""
    import torch

    p = W.quad6_problem(13)
    q = W.quad6_problem(13, dbar=(0.3, 0.3, 0.3))
    lt = torch.tensor(p.l, device=gpu)
    opts = __import__("paper_1903_07715_amd.hjr", fromlist=["x"]).problem_options(p, precision=hjrlib.FP32_POLISH64,
                                                                                 max_iter=20000)
    monkeypatch.setenv("HJR_NPT", "4")
    K = torch.empty_like(lt)
    hjrlib.solve_device(q.grid, q.dyn, lt, None, K, **opts)
    results = {}
    for cfg in ("4", "-1", "-8", "-16"):
        monkeypatch.setenv("HJR_NPT", cfg)
        for warm in (False, True):
            V = torch.empty_like(lt)
            r, st = hjrlib.solve_device(p.grid, p.dyn, lt, K if warm else None, V, **opts)
            print(f"[march] solve cfg={cfg} warm={warm}: {r['iterations']}+{r['polish_iterations']} status {st}",
                  flush=True)
            assert st == hjrlib.OK
            results[(cfg, warm)] = (r["iterations"], r["polish_iterations"], V.cpu())
    for cfg in ("-1", "-8", "-16"):
        for warm in (False, True):
            a, b = results[("4", warm)], results[(cfg, warm)]
            assert a[:2] == b[:2] and torch.equal(a[2], b[2])


def test_weno_march_solves_bitwise_equal_flat(gpu, hjrlib, monkeypatch):
    """Whole WENO5 + TVD-RK3 FP32 + FP64-polish solves of the 101^3 Dubins car, cold: the march
    configurations and the flat one give the same iterations and bitwise the same V."""
    import torch

    from paper_1903_07715_amd import hjr

    p = W.dubins_problem(101)
    lt = torch.tensor(p.l, device=gpu)
    opts = hjr.problem_options(p, precision=hjrlib.FP32_POLISH64, max_iter=20000)
    results = {}
    for cfg in ("4", "-4", "-1"):
        monkeypatch.setenv("HJR_NPT", cfg)
        V = torch.empty_like(lt)
        r, st = hjrlib.solve_device(p.grid, p.dyn, lt, None, V, **opts)
        print(f"[march] WENO5 solve cfg={cfg}: {r['iterations']}+{r['polish_iterations']} status {st}", flush=True)
        assert st == hjrlib.OK
        results[cfg] = (r["iterations"], r["polish_iterations"], V.cpu())
    for cfg in ("-4", "-1"):
        a, b = results["4"], results[cfg]
        assert a[:2] == b[:2] and torch.equal(a[2], b[2])
