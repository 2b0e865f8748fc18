"""GPU tests of the batched engine (many grids per launch) and the serving context
(continuous batching): each result is the same alone and in the mix, bitwise, because the
per-node arithmetic does not depend on which other instances share a launch."""
import time

import numpy as np
import pytest

from paper_1903_07715_amd import workloads as W

pytestmark = pytest.mark.gpu


def _mix():
    out = []
    for i, n in enumerate((31, 45, 61)):
        p = W.di_box_problem(n, ubar=0.8 + 0.2 * i, dbar=0.05 * i)
        p.spatial, p.temporal, p.cfl = 5, 3, 0.5
        out.append(p)
    for i, n in enumerate((21, 27, 33)):
        out.append(W.dubins_problem(n, ubar=1.0 + 0.25 * i, dbar=0.03 * i, center=(0.5 * i, -0.3 * i)))
    return out


def test_batch_alone_vs_mix_bitwise(gpu, hjrlib):
    probs = _mix()
    Vs, rs, sts = hjrlib.batch_solve([(p.grid, p.dyn) for p in probs], [p.l for p in probs], [None] * len(probs),
                                     [hjrlib.problem_options(p) for p in probs])
    for p, V, r, st in zip(probs, Vs, rs, sts):
        Va, ra, sta = hjrlib.solve(p.grid, p.dyn, p.l, None, **hjrlib.problem_options(p))
        assert st == sta == hjrlib.OK, p.name
        assert (r["iterations"], r["polish_iterations"]) == (ra["iterations"], ra["polish_iterations"]), p.name
        assert np.array_equal(V, Va), p.name


def test_batch_6d_bricks_alone_vs_mix_bitwise(gpu, hjrlib, monkeypatch):
    """6-D quadrotors of odd and even grid sizes batched through the brick plane-march kernel
    (each instance's bricks in one launch) give the results of their solves alone."""
    monkeypatch.setenv("HJR_NPT", "-16")
    probs = [W.quad6_problem(9, dbar=(0.5, 0.5, 0.5)), W.quad6_problem(10, dbar=(0.4, 0.3, 0.5)),
             W.quad6_problem(9, m=1.1, dbar=(0.3, 0.3, 0.3))]
    opts = [hjrlib.problem_options(p, max_iter=20000) for p in probs]
    Vs, rs, sts = hjrlib.batch_solve([(p.grid, p.dyn) for p in probs], [p.l for p in probs], [None] * len(probs), opts)
    for p, o, V, r, st in zip(probs, opts, Vs, rs, sts):
        Va, ra, sta = hjrlib.solve(p.grid, p.dyn, p.l, None, **o)
        print(f"[batch] {p.grid.n}: {r['iterations']}+{r['polish_iterations']} steps, status {st}", flush=True)
        assert st == sta == hjrlib.OK
        assert (r["iterations"], r["polish_iterations"]) == (ra["iterations"], ra["polish_iterations"])
        assert np.array_equal(V, Va)


def test_batch_matches_oracle(gpu, hjrlib, orc):
    probs = _mix()[1:5]
    Vs, rs, sts = hjrlib.batch_solve([(p.grid, p.dyn) for p in probs], [p.l for p in probs], [None] * len(probs),
                                     [hjrlib.problem_options(p) for p in probs])
    for p, V, st in zip(probs, Vs, sts):
        Vo, io = orc.solve(p.grid, p.dyn, p.l, max_iter=20000, **orc.problem_opts(p))
        assert io["converged"] == 1, p.name
        band = 1e-4 * np.abs(p.l).max()
        assert st == hjrlib.OK
        assert np.abs(V - Vo).max() <= band, p.name
        assert np.sum(((V <= 0) != (Vo <= 0)) & (np.abs(Vo) > band)) == 0


def test_batch64_every_instance_converges_and_subset_matches_oracle(gpu, hjrlib, orc):
    """The benchmark's 64-instance mixed batch (double integrator 51^2-201^2, Dubins 41^3-121^3,
    FP32, advanced together): every instance converges, and the smallest and largest double
    integrators and the two smallest and the largest Dubins grids match their FP64 oracle solves
    within the FP32 threshold's reach (8 FP32 spacings at max |l| per step; bar 1e-4 max|l|) with
    no off-band sign mismatch.  (The other Dubins grids equal their standalone solves bitwise by
    the alone-vs-mix tests.)"""
    probs = W.batch_problems(64)
    opts = [hjrlib.problem_options(p, precision=hjrlib.FP32, max_iter=20000) for p in probs]
    Vs, rs, sts = hjrlib.batch_solve([(p.grid, p.dyn) for p in probs], [p.l for p in probs], [None] * len(probs),
                                     opts)
    print(f"[batch64] statuses {sorted(set(sts))}, steps {min(r['iterations'] for r in rs)}.."
          f"{max(r['iterations'] for r in rs)}", flush=True)
    assert all(st == hjrlib.OK for st in sts), [p.name for p, st in zip(probs, sts) if st != hjrlib.OK]
    di = sorted((p.grid.n[0], i) for i, p in enumerate(probs) if p.grid.ndim == 2)
    du = sorted((p.grid.n[0], i) for i, p in enumerate(probs) if p.grid.ndim == 3)
    for _, i in (di[0], di[-1], du[0], du[1], du[-1]):
        p = probs[i]
        print(f"[batch64] oracle solve of {p.name} ...", flush=True)
        Vo, io = orc.solve(p.grid, p.dyn, p.l, max_iter=20000, **orc.problem_opts(p))
        assert io["converged"] == 1, p.name
        band = 1e-4 * np.abs(p.l).max()
        err = np.abs(Vs[i] - Vo).max()
        mism = int(np.sum(((Vs[i] <= 0) != (Vo <= 0)) & (np.abs(Vo) > band)))
        print(f"[batch64] {p.name}: max|V - V_oracle| {err:.3e} (bar {band:.3e}), mismatches {mism}", flush=True)
        assert err <= band and mism == 0


def test_batch_mixed_precision_and_schemes(gpu, hjrlib):
    """FP64, FP32 and FP32+polish instances, Euler and RK3, advance in the same launches."""
    p1 = W.di_box_problem(51)
    p2 = W.dubins_problem(25)
    p3 = W.di_box_problem(41, dbar=0.2)
    cases = [(p1, dict(precision=hjrlib.FP64, spatial=1, temporal=1, cfl=0.8)),
             (p2, dict(precision=hjrlib.FP32, **hjrlib.problem_options(p2))),
             (p3, dict(precision=hjrlib.FP32_POLISH64, spatial=1, temporal=1, cfl=0.8))]
    Vs, rs, sts = hjrlib.batch_solve([(p.grid, p.dyn) for p, _ in cases], [p.l for p, _ in cases], [None] * 3,
                                     [o for _, o in cases])
    for (p, o), V, r, st in zip(cases, Vs, rs, sts):
        Va, ra, sta = hjrlib.solve(p.grid, p.dyn, p.l, None, **o)
        assert st == sta and np.array_equal(V, Va), p.name


def _dev(torch, a, device):
    return torch.tensor(a, device=device)


def test_context_results_equal_alone(gpu, hjrlib):
    torch = __import__("torch")
    probs = _mix()
    ref = []
    for p in probs:
        V, r, st = hjrlib.solve(p.grid, p.dyn, p.l, None, **hjrlib.problem_options(p))
        ref.append((V, r))
    with hjrlib.Context(0) as ctx:
        tickets, outs = [], []
        for i, p in enumerate(probs):
            l_t = _dev(torch, p.l, gpu)
            V_t = torch.empty_like(l_t)
            torch.cuda.synchronize()
            tickets.append(ctx.submit(p.grid, p.dyn, l_t, None, V_t, **hjrlib.problem_options(p)))
            outs.append(V_t)
            time.sleep(0.002 * i)  # staggered arrivals: later requests join running ones
        done = {}
        deadline = time.time() + 120
        while len(done) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in done:
                    r = ctx.poll(t)
                    if r is not None:
                        done[t] = r
            time.sleep(0.001)
        assert len(done) == len(tickets)
        st = ctx.stats()
        assert st["admitted"] == st["finished"] == len(probs)
    for t, V_t, (Vr, rr) in zip(tickets, outs, ref):
        status, res = done[t]
        assert status == hjrlib.OK
        assert (res["iterations"], res["polish_iterations"]) == (rr["iterations"], rr["polish_iterations"])
        assert np.array_equal(V_t.cpu().numpy(), Vr)


def test_context_memory_budget(gpu, hjrlib):
    torch = __import__("torch")
    p = W.dubins_problem(41)
    l_t = _dev(torch, p.l, gpu)
    # one request needs 4 FP32 + 2 FP64 arrays plus tables: ~32 B per node
    budget = int(p.grid.size * 40)
    with hjrlib.Context(0, budget) as ctx:
        outs = [torch.empty_like(l_t) for _ in range(4)]
        ts = [ctx.submit(p.grid, p.dyn, l_t, None, V, **hjrlib.problem_options(p)) for V in outs]
        ctx.drain()
        stats = ctx.stats()
        assert stats["bytes_peak"] <= budget
        for t in ts:
            assert ctx.poll(t)[0] == hjrlib.OK
        for V in outs[1:]:
            assert torch.equal(V, outs[0])
        big = W.dubins_problem(81)
        lb = _dev(torch, big.l, gpu)
        with pytest.raises(hjrlib.HJRError) as e:
            ctx.submit(big.grid, big.dyn, lb, None, torch.empty_like(lb), **hjrlib.problem_options(big))
        assert e.value.status == hjrlib.ERR_BUDGET


def test_context_bad_request_does_not_disturb_others(gpu, hjrlib):
    torch = __import__("torch")
    good = W.dubins_problem(25)
    bad = W.dubins_problem(25)
    lbad = bad.l.copy()
    lbad[3, 4, 5] = np.nan
    Vref, _, _ = hjrlib.solve(good.grid, good.dyn, good.l, None, **hjrlib.problem_options(good))
    with hjrlib.Context(0) as ctx:
        lg, lb = _dev(torch, good.l, gpu), _dev(torch, lbad, gpu)
        Vg, Vb = torch.empty_like(lg), torch.empty_like(lb)
        tb = ctx.submit(bad.grid, bad.dyn, lb, None, Vb, **hjrlib.problem_options(bad))
        tg = ctx.submit(good.grid, good.dyn, lg, None, Vg, **hjrlib.problem_options(good))
        ctx.drain()
        assert ctx.poll(tb)[0] == hjrlib.ERR_NONFINITE
        assert ctx.poll(tg)[0] == hjrlib.OK
        assert np.array_equal(Vg.cpu().numpy(), Vref)


def test_warm_start_server_results_against_oracle(gpu, hjrlib, orc):
    """The serving loop's warm-start policy (serving.WarmStartServer) over a short stream of
    double-integrator and Dubins requests whose control and disturbance bounds change.  Each
    request is warm-started from the nearest converged prior of its kind, preferring one whose
    problem dominates it (more control authority, no more disturbance).  A dominating prior
    gives the new problem's value function exactly (Theorem 2 with Prop. 2): the result matches
    the cold FP64 oracle solve within 1e-4 max|l| with no off-band sign mismatch.  Any other
    prior is conservative (Theorem 1): every node the oracle puts in the unsafe set off the band
    is unsafe in the result too.  Requests arrive one after another, so the prior each one sees
    is fixed."""
    import torch

    from paper_1903_07715_amd import serving

    di = W.di_box_problem(61)
    du = W.dubins_problem(41, scheme="upwind")
    kinds = {"di2": (di, torch.tensor(di.l, device=gpu)), "dubins3": (du, torch.tensor(du.l, device=gpu))}
    dom = lambda a, b: a[0] <= b[0] and a[1] <= b[1]  # key = (-control bound, disturbance bound)
    params = [("di2", 1.2, 0.05), ("dubins3", 1.6, 0.05), ("di2", 1.0, 0.10), ("dubins3", 1.2, 0.12),
              ("di2", 1.4, 0.02), ("dubins3", 1.8, 0.02), ("di2", 0.9, 0.12), ("dubins3", 1.0, 0.15)]
    reqs = []
    for j, (kind, ub, db) in enumerate(params):
        p, lt = kinds[kind]
        dyn = W.double_integrator(ub, 1.0, db) if kind == "di2" else W.dubins3(1.0, ub, db)
        opts = hjrlib.problem_options(p, precision=hjrlib.FP32_POLISH64, max_iter=20000)
        reqs.append(serving.Request(kind=kind, grid=p.grid, dyn=dyn, key=(-ub, db), dominates=dom, l_dev=lt,
                                    opts=opts, arrival=0.6 * j))
    with hjrlib.Context(0) as ctx:
        serving.WarmStartServer(ctx, warm=True).run(reqs, torch, gpu)
    n_exact = n_cons = 0
    for r in reqs:
        p = kinds[r.kind][0]
        assert r.status == hjrlib.OK, (r.kind, r.key)
        V = r.V.cpu().numpy().reshape(p.grid.shape)
        Vo, io = orc.solve(p.grid, r.dyn, p.l, **orc.problem_opts(p))
        assert io["converged"] == 1
        band = 1e-4 * float(np.abs(p.l).max())
        err = float(np.abs(V - Vo).max())
        print(f"[serve] {r.kind} key {r.key} warm from {r.warm_from} exact={r.exact_warm}: "
              f"max|V - V_oracle| {err:.3e} (bar {band:.3e})", flush=True)
        if r.exact_warm is None or r.exact_warm:
            n_exact += r.exact_warm is not None
            assert err <= band
            assert np.sum(((V <= 0) != (Vo <= 0)) & (np.abs(Vo) > band)) == 0
        else:
            n_cons += 1
            assert not np.any((Vo < -band) & (V > 0))       # the unsafe set only grows
            assert (V - Vo).max() <= band                    # V_k <= V_l up to the tolerance
    assert n_exact >= 2 and n_cons >= 2, (n_exact, n_cons)
