"""Benchmark: warm-started HJI reachability solves on one MI355X.

One benchmark step is one complete warm-started solve of the 6-D quadrotor (translational
dynamics, thrust and two tilt angles as controls, a disturbance on every acceleration) on a 25^6
grid (244 M nodes, p in [-5,5]^3, v in [-3,3]^3, a cube obstacle |p_i| <= 1): first-order upwind +
Lax-Friedrichs + forward Euler at CFL 0.8 in FP32 until the max-norm change is below the FP32
threshold, then the FP64 polish to 1e-6.  The warm start k is the solution with the smaller
disturbance bound 0.3 (the new problem has 0.5; exact by Theorem 2).  Inputs (l, k) are resident
in device memory before the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload quad6|dubins|...]

Prints one JSON line.  `value` is grid-point updates per second over the timed solves (every
node advanced one full time step, FP32 and FP64 steps alike).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 operations per node per stage of the WENO5 + Lax-Friedrichs operator on the
# Dubins car, counted from the scheme's definition (each add, multiply, abs, max, reciprocal = 1):
#   per dimension: 6 first differences (6 sub + 6 scale) = 12; two WENO5 derivatives at 84 each
#   (candidates 15, second differences 9, third-order terms 9, smoothness 15, eps 11, weights 17,
#   combination 8) = 168; average and jump of D-/D+ = 4                       -> 184 per dim
#   Hamiltonian with dissipation coefficients = 20; dissipation sum = 6; stage combination = 5
FLOP_PER_NODE_STAGE_DUBINS_WENO5 = 3 * 184 + 20 + 6 + 5          # = 583
# Algorithmic HBM bytes per node per RK3 step in FP32 (no halo re-reads): stage 1 reads V, writes
# V1 (8); stage 2 reads V1, V, writes V2 (12); stage 3 reads V2, V, l, writes V (16).
BYTES_PER_NODE_STEP_RK3_FP32 = 36
# One forward-Euler step reads V and l and writes V: 12 bytes per node in FP32, 24 in FP64.
BYTES_PER_NODE_STEP_EULER_FP32 = 12
BYTES_PER_NODE_STEP_EULER_FP64 = 24

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (packed FMA) peak
PEAK_HBM_GBS = 8000.0

# Bytes per launch of the headline's FP32 stage kernel (the brick plane-march kernel on the 25^6
# quadrotor) between L2 and memory, from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a
# 1 GiB copy calibration (profiles/quad6_25_headline_hbm_counters.txt), keyed by a hash of the
# kernel sources they were taken from: a kernel changed since then reports null.
MEASURED_TRAFFIC = {"22dc968893426f53": {"quad6": 4.092e9 + 1.007e9}}


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("hjr_device.hpp", "hjr_kernels.hip"):
        with open(os.path.join(ROOT, "paper_1903_07715_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def tuner_config(fp64: bool, dyn_id: int, spatial: int, nodes: int):
    """The launch configuration the library uses for a group of this size class: HJR_NPT when
    set, else the tuner's choice from its cache file (HJR_TUNE_CACHE, which main() points at a
    fresh file unless the caller set one), or None before the tuner has chosen."""
    if os.environ.get("HJR_NPT"):
        return int(os.environ["HJR_NPT"])
    path = os.environ.get("HJR_TUNE_CACHE")
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        choices = json.load(f)
    key = f"fp{64 if fp64 else 32}_dyn{dyn_id}_sp{spatial}_n2^{int(nodes).bit_length() - 1}"
    for k, v in choices.items():
        if k == key or k.startswith(key + "_"):
            return int(v)
    return None


def kernel_name(cfg, fp64: bool, model: str, scheme: str = "upwind"):
    t = "double" if fp64 else "float"
    if cfg == -16:
        return f"march_brick_kernel<{t}, {model}> (2 x 2 x 2 row bricks, whole lines)"
    if cfg is not None and cfg < 0:
        return f"march_kernel<{t}, {model}> ({'whole lines' if cfg == -1 else f'runs of {-cfg} planes'})"
    if cfg:
        return f"stage_kernel_one<{t}, {model}, {scheme}, {cfg} nodes per thread>"
    return "the stage kernel the tuner keeps"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=101, help="grid side (default 101)")
    ap.add_argument("--polish-shift", type=float, default=-1.0, help="FP64 polish start shift (< 0: automatic)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["quad6", "dubins", "unicycle", "batch", "serve", "control", "quad10", "hbm",
                                           "discount", "local", "warmcold"],
                    default="quad6",
                    help="quad6: the headline, warm-started FP32 + FP64-polish solves of the 25^6 quadrotor; "
                         "dubins: warm-started solves of the 101^3 Dubins car (WENO5 + TVD-RK3); "
                         "unicycle: the 61^4 unicycle after one of its two obstacles moves, cold vs warm; "
                         "batch: the 64-instance mixed batch; "
                         "serve: a Poisson request stream through the serving context, warm vs cold; "
                         "control: safe-control queries against the converged 101^3 Dubins value function; "
                         "quad10: the 10-D near-hover quadrotor scenario of Sec. VI by subsystem, warm vs cold; "
                         "hbm: FP32 upwind + Euler steps of the 25^6 quadrotor (the HBM-bound path); "
                         "discount: standard vs warm-started vs discounted solves (Table 1's comparison); "
                         "local: warm-started solves after a local change of the environment, with and "
                         "without local updates; "
                         "warmcold: warm vs cold steps and time under the per-step rule (FP32 threshold at 3 "
                         "and 8 spacings) and the interval rule of Sec. IV")
    ap.add_argument("--discount", type=float, default=None,
                    help="discount: per-step factor, annealed to 1 (default: Table 1's 0.999)")
    ap.add_argument("--queries", type=int, default=1 << 20, help="control: query states per batch")
    ap.add_argument("--requests", type=int, default=256, help="serve: number of requests")
    ap.add_argument("--serve-budget-gb", type=int, default=128, help="serve: HBM budget of the serving context")
    ap.add_argument("--serve-in-flight", type=int, default=24, help="serve: requests submitted and not yet done")
    ap.add_argument("--quad-n", type=int, default=25, help="quad6, hbm, serve: grid side of the 6-D quadrotor")
    ap.add_argument("--parity-n", type=int, default=9,
                    help="quad6: grid side of the reduced solve the CPU-baseline leg also checks against")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, run 5 plain device copies of MIB MiB (HBM counter calibration)")
    return ap.parse_args()


def copy_calibration(mib):
    """Plain device-to-device copies of a known size, to scale the HBM byte counters."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read_per_copy": n * 4, "bytes_written_per_copy": n * 4, "copies": 5}),
          flush=True)


def cpu_baseline(p, npts, seconds):
    """The FP64 oracle, as it stands, timed on the host: full TVD-RK3 steps of the same grid."""
    import numpy as np

    import oracle

    opts = oracle.problem_opts(p)
    dt = oracle.cfl_dt(p.grid, p.dyn, p.cfl)
    V = p.l.copy()
    t0 = time.perf_counter()
    steps = 0
    while True:
        V, _ = oracle.step(p.grid, p.dyn, V, p.l, dt, spatial=opts["spatial"], temporal=opts["temporal"])
        steps += 1
        log(f"  oracle step {steps}: {time.perf_counter() - t0:.1f} s")
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    assert np.all(np.isfinite(V))
    return {"value": steps * npts / el, "unit": "grid-point updates/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{steps} FP64 WENO5+TVD-RK3 steps of the {p.grid.n[0]}^3 Dubins grid from V=l "
                      f"({el:.1f} s)"}


def main():
    args = parse()
    if not os.environ.get("HJR_TUNE_CACHE"):
        import tempfile

        os.environ["HJR_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="hjr_tune_"), "choices.json")
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.workload == "control":
        return bench_control(args)
    if args.workload == "quad10":
        return bench_quad10(args)
    if args.workload == "hbm":
        return bench_hbm(args)
    if args.workload == "discount":
        return bench_discount(args)
    if args.workload == "local":
        return bench_local(args)
    if args.workload == "warmcold":
        return bench_warmcold(args)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload == "quad6":
        return bench_quad6(args)
    if args.workload == "unicycle":
        return bench_unicycle(args)
    return bench_dubins(args)


def working_avg(entries):
    """Average event-timed duration (s) of the working launches (steps some instance was still
    taking; launches issued after convergence return at once and are left out)."""
    n = sum(e["working_launches"] for e in entries)
    ms = sum(e["working_ms"] for e in entries)
    return (ms / n / 1e3 if n else float("nan")), n


def cpu_baseline_quad6(p, q, n_par, gpu_solve):
    """The FP64 oracle, as it stands, on the host: the same warm-started problem on a reduced
    n^6 grid (its prior solve, then the warm-started solve, which is timed).  The GPU solves the
    same reduced problem from the oracle's prior, and the two results are compared: max |V - V_oracle|
    and the nodes whose sign differs where |V_oracle| > 1e-4 max|l|."""
    import numpy as np

    import oracle
    from paper_1903_07715_amd import workloads as W

    pr = W.quad6_problem(n_par, m=p.dyn.params[1], dbar=p.dyn.params[6:9])
    qr = W.quad6_problem(n_par, m=q.dyn.params[1], dbar=q.dyn.params[6:9])
    opts = oracle.problem_opts(pr)
    t0 = time.perf_counter()
    K, ik = oracle.solve(qr.grid, qr.dyn, qr.l, **opts)
    t1 = time.perf_counter()
    log(f"  oracle prior {n_par}^6: {ik['steps']} steps, {t1 - t0:.1f} s")
    V, iv = oracle.solve(pr.grid, pr.dyn, pr.l, K, **opts)
    t2 = time.perf_counter()
    log(f"  oracle warm {n_par}^6: {iv['steps']} steps, {t2 - t1:.1f} s")
    Vg, st, res = gpu_solve(pr, K)
    band = 1e-4 * float(np.abs(pr.l).max())
    err = float(np.abs(Vg - V).max())
    mism = int(np.sum(((Vg <= 0) != (V <= 0)) & (np.abs(V) > band)))
    base = {"value": iv["steps"] * pr.grid.size / (t2 - t1), "unit": "grid-point updates/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"the warm-started solve of the same problem on a {n_par}^6 grid ({iv['steps']} FP64 "
                      f"upwind + Euler steps, {t2 - t1:.1f} s; its prior solve took {t1 - t0:.1f} s more)"}
    parity = {"grid": [n_par] * 6, "max_abs_err": err, "band": band, "err_over_band": err / band,
              "sign_mismatches_off_band": mism, "gpu_status": st,
              "gpu_steps": [res["iterations"], res["polish_iterations"]], "oracle_steps": iv["steps"]}
    return base, parity


def bench_quad6(args):
    """The headline: warm-started FP32 + FP64-polish solves of the 6-D quadrotor on a 25^6 grid."""
    import numpy as np
    import torch

    from paper_1903_07715_amd import hjr
    from paper_1903_07715_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    n = args.quad_n
    p = W.quad6_problem(n, m=1.2, dbar=(0.5, 0.5, 0.5))
    q = W.quad6_problem(n, m=1.2, dbar=(0.3, 0.3, 0.3))
    npts = p.grid.size
    opts = hjr.problem_options(p, precision=hjr.FP32_POLISH64, max_iter=20000, polish_shift=args.polish_shift)
    stream = torch.cuda.Stream()
    l_t = torch.tensor(p.l, device=dev)
    k_t = torch.empty_like(l_t)
    V_t = torch.empty_like(l_t)
    log(f"quad6 {n}^6 = {npts} nodes; warm-start function: the solution with disturbance 0.3")
    rq, sq = hjr.solve_device(q.grid, q.dyn, l_t, None, k_t, stream=stream, **opts)
    torch.cuda.synchronize()
    log(f"  prior: {rq['iterations']}+{rq['polish_iterations']} steps, status {sq}, {rq['seconds']:.3f} s")

    def run(warm: bool):
        return hjr.solve_device(p.grid, p.dyn, l_t, k_t if warm else None, V_t, stream=stream, **opts)

    for i in range(args.warmup):
        r, st = run(True)
        log(f"warmup {i}: {r['iterations']}+{r['polish_iterations']} steps, status {st}, {r['seconds']:.3f} s")
    # the tuner times each candidate launch configuration on a chunk of steps; a solve has only a
    # few FP64 polish steps, so its FP64 search may need more solves than the warm-up: finish it
    # untimed, so the timed solves run with the configurations it settled on
    for i in range(12):
        if tuner_config(False, p.dyn.id, 1, npts) is not None and tuner_config(True, p.dyn.id, 1, npts) is not None:
            break
        r, st = run(True)
        log(f"tuning solve {i}: {r['iterations']}+{r['polish_iterations']} steps, status {st}, {r['seconds']:.3f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates = 0
    statuses = []
    res = None
    for i in range(args.steps):
        res, st = run(True)
        statuses.append(st)
        updates += (res["iterations"] + res["polish_iterations"]) * npts
        log(f"timed warm solve {i}: {res['iterations']}+{res['polish_iterations']} steps, status {st}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    # the same solves with launch-stamped events around every stage kernel (kept out of `value`)
    hjr.profile_read(reset=True)
    hjr.profile_enable(True)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for i in range(args.steps):
        run(True)
    torch.cuda.synchronize()
    pel = time.perf_counter() - p0
    hjr.profile_enable(False)
    prof = hjr.profile_read(reset=True)
    log(f"event-timed pass: {pel:.3f} s vs {el:.3f} s untimed")

    torch.cuda.synchronize()
    c0 = time.perf_counter()
    cres = None
    cstat = []
    for i in range(args.steps):
        cres, cst = run(False)
        cstat.append(cst)
        log(f"cold solve {i}: {cres['iterations']}+{cres['polish_iterations']} steps, status {cst}")
    torch.cuda.synchronize()
    cel = time.perf_counter() - c0

    # one warm solve through the host-array entry point (l and k in over PCIe, V back)
    l_h = p.l
    k_h = k_t.cpu().numpy().reshape(p.grid.shape)
    h0 = time.perf_counter()
    hjr.solve(p.grid, p.dyn, l_h, k_h, **opts)
    hel = time.perf_counter() - h0
    log(f"host-array warm solve: {hel:.3f} s")
    del k_h

    avg32, n32 = working_avg(prof["stage32"])
    avg64, n64 = working_avg(prof["stage64"])
    gbs32 = BYTES_PER_NODE_STEP_EULER_FP32 * npts / avg32 / 1e9
    gbs64 = BYTES_PER_NODE_STEP_EULER_FP64 * npts / avg64 / 1e9
    roofline = {"bound": "hbm", "achieved": round(gbs32, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs32 / PEAK_HBM_GBS, 4),
                "traffic": MEASURED_TRAFFIC.get(kernel_source_hash(), {}).get("quad6") if n == 25 else None,
                "kernel": kernel_name(tuner_config(False, p.dyn.id, 1, npts), False, "Quad6")
                + ": upwind + Lax-Friedrichs + Euler step, FP32",
                "bytes_per_update": BYTES_PER_NODE_STEP_EULER_FP32,
                "avg_launch_us": round(avg32 * 1e6, 1), "working_launches": n32,
                "fp64_polish_kernel": {"kernel": kernel_name(tuner_config(True, p.dyn.id, 1, npts), True, "Quad6"),
                                       "achieved": round(gbs64, 1), "frac": round(gbs64 / PEAK_HBM_GBS, 4),
                                       "bytes_per_update": BYTES_PER_NODE_STEP_EULER_FP64,
                                       "avg_launch_us": round(avg64 * 1e6, 1), "working_launches": n64}}
    line = {
        "metric": "grid-point updates/s (%HBM peak); warm vs cold solves/s, p50/p99 latency",
        "value": updates / el,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"quad6-{n}^6-upwind-euler-fp32-polish64-warm", "grid": [n] * 6, "points": npts,
                   "cfl": p.cfl, "tol": p.tol, "mass": 1.2, "dbar": 0.5, "prior_dbar": 0.3},
        "ms_per_solve": el / args.steps * 1e3,
        "warm_solves_per_s": args.steps / el,
        "cold_solves_per_s": args.steps / cel,
        "warm_over_cold": cel / el,
        "warm_iterations": [res["iterations"], res["polish_iterations"]],
        "cold_iterations": [cres["iterations"], cres["polish_iterations"]],
        "statuses_warm": statuses,
        "statuses_cold": cstat,
        "host_io_warm_solves_per_s": 1.0 / hel,
        "event_pass_seconds": pel,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) and reduced-grid parity")

        def gpu_solve(pr, K):
            lt = torch.tensor(pr.l, device=dev)
            kt = torch.tensor(K, device=dev)
            Vt = torch.empty_like(lt)
            r, st = hjr.solve_device(pr.grid, pr.dyn, lt, kt, Vt, **hjr.problem_options(
                pr, precision=hjr.FP32_POLISH64, max_iter=20000))
            torch.cuda.synchronize()
            return Vt.cpu().numpy().reshape(pr.grid.shape), st, r

        line["cpu_baseline"], line["parity"] = cpu_baseline_quad6(p, q, args.parity_n, gpu_solve)
    print(json.dumps(line), flush=True)


def bench_unicycle(args):
    """The 4-D unicycle on 61^4 (13.8 M nodes) among two seeded disks; one disk moves by 0.3 and
    the value function is recomputed cold and warm-started from the one before the move (neither
    obstacle set contains the other, so Theorem 1 promises only a conservative result: the warm
    unsafe set contains the cold one).  First-order upwind + Euler, FP32 + FP64 polish, solved to
    convergence (WENO5 + TVD-RK3, the configuration's scheme, has no steady state here; its
    fixed-step parity is tested).  Reports steps, statuses, solves/s and the set containment."""
    import numpy as np
    import torch

    from paper_1903_07715_amd import hjr
    from paper_1903_07715_amd import workloads as W

    dev = torch.device("cuda:0")
    old = W.unicycle_problem(61)
    new = W.unicycle_problem(61, moved=True)
    for p in (old, new):
        p.spatial, p.temporal, p.cfl = 1, 1, 0.8
    opts = hjr.problem_options(new, precision=hjr.FP32_POLISH64, max_iter=100000)
    lo, ln = torch.tensor(old.l, device=dev), torch.tensor(new.l, device=dev)
    K = torch.empty_like(lo)
    r0, s0 = hjr.solve_device(old.grid, old.dyn, lo, None, K, **opts)
    log(f"unicycle 61^4 before the move: {r0['iterations']}+{r0['polish_iterations']} steps, status {s0}")
    out = {"workload": "unicycle4-61^4-two-disks-move0.3-upwind-euler-fp32-polish64", "nodes": new.grid.size,
           "prior": {"steps": [r0["iterations"], r0["polish_iterations"]], "status": s0, "seconds": r0["seconds"]}}
    Vs = {}
    for warm in (False, True):
        V = torch.empty_like(ln)
        hjr.solve_device(new.grid, new.dyn, ln, K if warm else None, V, **opts)  # untimed (tuning)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r, st = hjr.solve_device(new.grid, new.dyn, ln, K if warm else None, V, **opts)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / args.steps
        Vs[warm] = V.cpu().numpy()
        key = "warm" if warm else "cold"
        out[key] = {"seconds": el, "solves_per_s": 1.0 / el, "steps": [r["iterations"], r["polish_iterations"]],
                    "status": st}
        log(f"{key}: {out[key]}")
    band = 1e-4 * float(np.abs(new.l).max())
    out["warm_over_cold"] = out["cold"]["seconds"] / out["warm"]["seconds"]
    out["max_abs_warm_minus_cold"] = float(np.abs(Vs[True] - Vs[False]).max())
    out["cold_unsafe_nodes_not_unsafe_warm"] = int(np.sum((Vs[False] < -band) & (Vs[True] > 0)))
    out["unsafe_nodes"] = {"cold": int(np.sum(Vs[False] <= 0)), "warm": int(np.sum(Vs[True] <= 0))}
    print(json.dumps(out), flush=True)


def bench_dubins(args):
    import torch

    from paper_1903_07715_amd import hjr
    from paper_1903_07715_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    n = args.n
    p = W.dubins_problem(n, dbar=0.1)
    q = W.dubins_problem(n, dbar=0.05)
    npts = p.grid.size
    opts = hjr.problem_options(p, precision=hjr.FP32_POLISH64, max_iter=20000, polish_shift=args.polish_shift)
    stream = torch.cuda.Stream()
    l_t = torch.tensor(p.l, device=dev)
    lq_t = torch.tensor(q.l, device=dev)
    k_t = torch.empty_like(l_t)
    V_t = torch.empty_like(l_t)
    # warm-start function: the GPU solution of the smaller-disturbance problem
    log(f"warm-start function: solving {q.name} (dbar 0.05)")
    rq, _ = hjr.solve_device(q.grid, q.dyn, lq_t, None, k_t, stream=stream,
                             **dict(opts, precision=hjr.FP64))
    torch.cuda.synchronize()
    log(f"  done: {rq['iterations']}+{rq['polish_iterations']} steps in {rq['seconds']:.3f} s")

    def run(warm: bool):
        return hjr.solve_device(p.grid, p.dyn, l_t, k_t if warm else None, V_t, stream=stream, **opts)

    for i in range(args.warmup):
        r, _ = run(True)
        log(f"warmup {i}: {r['iterations']}+{r['polish_iterations']} steps in {r['seconds']:.3f} s")
    torch.cuda.synchronize()

    # timed region: warm solves
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates = 0
    res = None
    for i in range(args.steps):
        res, st = run(True)
        updates += (res["iterations"] + res["polish_iterations"]) * npts
        log(f"timed warm solve {i}: {res['iterations']}+{res['polish_iterations']} steps, status {st}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    # the same solves again with a HIP event pair around every stage-kernel launch, for the
    # kernel's average launch duration (the events themselves slow the step loop a little, so
    # they are kept out of the region `value` is measured on)
    hjr.profile_read(reset=True)
    hjr.profile_enable(True)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for i in range(args.steps):
        run(True)
    torch.cuda.synchronize()
    pel = time.perf_counter() - p0
    hjr.profile_enable(False)
    prof = hjr.profile_read(reset=True)
    log(f"event-timed pass: {pel:.3f} s vs {el:.3f} s untimed")

    # cold solves on the same problem, for the warm/cold comparison (not part of `value`)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    cres = None
    for i in range(args.steps):
        cres, _ = run(False)
        log(f"cold solve {i}: {cres['iterations']}+{cres['polish_iterations']} steps")
    torch.cuda.synchronize()
    cel = time.perf_counter() - c0

    # the same warm solves through the host-array entry point: l and k go over PCIe in and V
    # comes back each time (reported beside `value`, never as it)
    k_h = k_t.cpu().numpy().reshape(p.grid.shape)
    hjr.solve(p.grid, p.dyn, p.l, k_h, **opts)
    h0 = time.perf_counter()
    for i in range(args.steps):
        hjr.solve(p.grid, p.dyn, p.l, k_h, **opts)
    hel = time.perf_counter() - h0
    log(f"host-array warm solves: {hel / args.steps * 1e3:.1f} ms each")

    avg_s, launches = working_avg(prof["stage32"])
    flops = FLOP_PER_NODE_STAGE_DUBINS_WENO5 * npts
    achieved_tflops = flops / avg_s / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4),
                "traffic": MEASURED_TRAFFIC.get(kernel_source_hash(), {}).get("dubins") if n == 101 else None,
                "kernel": "the FP32 WENO5 + LF + TVD-RK3 stage kernel the tuner keeps (flat tiles or the march kernel)",
                "avg_launch_us": round(avg_s * 1e6, 2), "working_launches": launches,
                "algorithmic_gbs": round(BYTES_PER_NODE_STEP_RK3_FP32 / 3 * npts / avg_s / 1e9, 1)}
    line = {
        "metric": "grid-point updates/s (warm-started solve)",
        "value": updates / el,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"dubins3d-{n}^3-weno5-tvdrk3-fp32-polish64-warm", "grid": [n, n, n],
                   "points": npts, "cfl": p.cfl, "tol": p.tol},
        "warm_solves_per_s": args.steps / el,
        "event_pass_seconds": pel,
        "cold_solves_per_s": args.steps / cel,
        "host_io_warm_solves_per_s": args.steps / hel,
        "warm_iterations": [res["iterations"], res["polish_iterations"]],
        "cold_iterations": [cres["iterations"], cres["polish_iterations"]],
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(p, npts, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def bench_warmcold(args):
    """Warm vs cold under each stopping rule: per-step max-change below 1e-6 (FP32 + polish with
    the FP32 threshold at 3 and at 8 FP32 spacings of max |l|), and the interval rule of Sec. IV
    (change over an interval of 0.01 below 1e-3).  101^3 Dubins (WENO5 + TVD-RK3, FP32 + polish,
    warm from the |d_i| <= 0.05 solution: Theorem 2's exact case) and the 101^2 double
    integrator (upwind + Euler, FP64, warm from the |u| <= 0.8 solution: Remark 2's conservative
    case).  Each solve runs once untimed, then once timed."""
    import numpy as np
    import torch

    from paper_1903_07715_amd import hjr
    from paper_1903_07715_amd import workloads as W

    dev = torch.device("cuda:0")
    cases = [("dubins3d-101^3-weno5-tvdrk3-fp32-polish64", W.dubins_problem(101, dbar=0.1),
              W.dubins_problem(101, dbar=0.05), hjr.FP32_POLISH64),
             ("double-integrator-101^2-upwind-euler-fp64", W.di_box_problem(101, ubar=1.0),
              W.di_box_problem(101, ubar=0.8), hjr.FP64)]
    out = {}
    for name, p, q, prec in cases:
        lt, lq = torch.tensor(p.l, device=dev), torch.tensor(q.l, device=dev)
        kt, Vt = torch.empty_like(lt), torch.empty_like(lt)
        hjr.solve_device(q.grid, q.dyn, lq, None, kt, **hjr.problem_options(q, precision=hjr.FP64, max_iter=200000))
        spacing = 2.0 ** (math.frexp(float(np.abs(p.l).max()))[1] - 24)
        rules = {"per_step_1e-6": dict(tol=1e-6)}
        if prec == hjr.FP32_POLISH64:
            rules["per_step_1e-6_fp32_at_8_spacings"] = dict(tol=1e-6, tol_fp32=max(1e-6, 8 * spacing))
        rules["interval_0.01_1e-3"] = dict(tol=1e-3, conv_mode=hjr.CONV_PER_INTERVAL, dt_report=0.01)
        res = {}
        for rname, extra in rules.items():
            row = {}
            for warm in (False, True):
                opts = hjr.problem_options(p, precision=prec, max_iter=200000, **extra)
                for _ in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    r, st = hjr.solve_device(p.grid, p.dyn, lt, kt if warm else None, Vt, **opts)
                    torch.cuda.synchronize()
                    el = time.perf_counter() - t0
                row["warm" if warm else "cold"] = {"steps": [r["iterations"], r["polish_iterations"]],
                                                   "intervals": r["intervals"], "seconds": el, "status": st}
            row["warm_over_cold_seconds"] = row["warm"]["seconds"] / row["cold"]["seconds"]
            res[rname] = row
            log(f"{name} {rname}: {row}")
        out[name] = res
    print(json.dumps({"workload": "warm-vs-cold", "results": out}), flush=True)


def bench_discount(args):
    """Table 1's comparison on two of our problems: standard reachability (from l), warm start
    (from the solution of a smaller-disturbance problem, exact by Theorem 2) and discounted
    reachability (Sec. II-C, per-step factor annealed to 1), from l and from the same warm start.
    Each solve runs once untimed, then once timed; steps and device seconds are reported."""
    import numpy as np
    import torch

    from paper_1903_07715_amd import hjr
    from paper_1903_07715_amd import workloads as W

    dev = torch.device("cuda:0")
    if args.discount is None:
        args.discount = W.TABLE1_DISCOUNT
    out = {}
    probs = [("dubins3d-%d^3-weno5-tvdrk3-fp32-polish64" % args.n, W.dubins_problem(args.n, dbar=0.1),
              W.dubins_problem(args.n, dbar=0.05), dict(precision=hjr.FP32_POLISH64)),
             ("double-integrator-101^2-upwind-euler-fp64", W.di_box_problem(101, ubar=1.0, dbar=0.1),
              W.di_box_problem(101, ubar=1.0, dbar=0.05), dict(precision=hjr.FP64))]
    for name, p, q, extra in probs:
        opts = hjr.problem_options(p, max_iter=200000, **extra)
        lt, lq = torch.tensor(p.l, device=dev), torch.tensor(q.l, device=dev)
        kt, Vt = torch.empty_like(lt), torch.empty_like(lt)
        hjr.solve_device(q.grid, q.dyn, lq, None, kt, **dict(opts, precision=hjr.FP64))
        runs = {"standard": (None, 0.0), "warm": (kt, 0.0), "discounted": (None, args.discount),
                "discounted_warm": (kt, args.discount)}
        res = {}
        V = {}
        for key, (k, gamma) in runs.items():
            for timed in (False, True):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r, st = hjr.solve_device(p.grid, p.dyn, lt, k, Vt, **dict(opts, discount=gamma))
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
            V[key] = Vt.cpu().numpy()
            res[key] = {"seconds": el, "steps": r["iterations"] + r["polish_iterations"],
                        "discounted_steps": r["discounted_iterations"], "status": st}
            log(f"{name} {key}: {res[key]}")
        for key in ("warm", "discounted", "discounted_warm"):
            res[key]["max_abs_diff_vs_standard"] = float(np.abs(V[key] - V["standard"]).max())
            res[key]["unsafe_set_mismatch_nodes"] = int(np.sum((V[key] <= 0) != (V["standard"] <= 0)))
        res["discounted_over_warm_steps"] = res["discounted"]["steps"] / res["warm"]["steps"]
        res["discounted_over_warm_seconds"] = res["discounted"]["seconds"] / res["warm"]["seconds"]
        res["standard_over_warm_seconds"] = res["standard"]["seconds"] / res["warm"]["seconds"]
        out[name] = res
    print(json.dumps({"workload": "standard-vs-warm-vs-discounted", "discount": args.discount, "problems": out}),
          flush=True)


def bench_local(args):
    """Local updates (Sec. VII): the 101^3 Dubins value function is known; a small obstacle
    appears (a disk of radius 0.5 at (3, 3)), and the new value function is warm-started from
    the old one, once updating every node each step and once with local updates (bitwise the
    same result).  The new-obstacle problem uses first-order upwind + Euler: with a second,
    off-centre obstacle WENO5 + TVD-RK3 has no steady state (its iterates keep circulating, in
    FP64 and in the oracle alike).  Also the headline warm start (a global change: the
    disturbance bound, WENO5) both ways.  Each solve runs once untimed, then `--steps` times
    timed; statuses are reported, and every solve must converge."""
    import numpy as np
    import torch

    from paper_1903_07715_amd import hjr
    from paper_1903_07715_amd import workloads as W

    dev = torch.device("cuda:0")
    n = args.n
    p = W.dubins_problem(n, dbar=0.1)
    q = W.dubins_problem(n, dbar=0.05)
    opts = hjr.problem_options(p, precision=hjr.FP32_POLISH64, max_iter=20000)
    lt = torch.tensor(p.l, device=dev)
    V0 = torch.empty_like(lt)
    hjr.solve_device(p.grid, p.dyn, lt, None, V0, **opts)
    kq = torch.empty_like(lt)
    hjr.solve_device(q.grid, q.dyn, torch.tensor(q.l, device=dev), None, kq, **dict(opts, precision=hjr.FP64))
    pu = W.dubins_problem(n, dbar=0.1, scheme="upwind")
    uopts = hjr.problem_options(pu, precision=hjr.FP32_POLISH64, max_iter=20000)
    U0 = torch.empty_like(lt)
    hjr.solve_device(pu.grid, pu.dyn, lt, None, U0, **uopts)
    l2 = torch.tensor(np.minimum(p.l, W.disk_sdf(p.grid, (3.0, 3.0), 0.5)), device=dev)
    scen = {"new-obstacle-upwind": (l2, U0, uopts), "disturbance-change-weno5": (lt, kq, opts)}
    out = {}
    for name, (l, k, o) in scen.items():
        res = {}
        Vs = {}
        for local in (0, 1):
            Vt = torch.empty_like(lt)
            r, st = hjr.solve_device(p.grid, p.dyn, l, k, Vt, local_updates=local, **o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                r, st = hjr.solve_device(p.grid, p.dyn, l, k, Vt, local_updates=local, **o)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / args.steps
            Vs[local] = Vt.cpu().numpy()
            key = "local" if local else "full"
            res[key] = {"seconds": el, "steps": [r["iterations"], r["polish_iterations"]],
                        "node_updates": r["node_updates"], "status": st}
            log(f"{name} {key}: {res[key]}")
        res["bitwise_equal"] = bool(np.array_equal(Vs[0], Vs[1]))
        res["computed_fraction"] = res["local"]["node_updates"] / res["full"]["node_updates"]
        res["speedup"] = res["full"]["seconds"] / res["local"]["seconds"]
        out[f"dubins{n}^3-fp32-polish64 {name}"] = res
    # the double integrator, upwind + Euler in FP64 (a reach of one node per step), 1001^2
    d = W.di_box_problem(1001, ubar=1.0, dbar=0.1)
    dopt = dict(spatial=1, temporal=1, cfl=0.8, tol=1e-6, precision=hjr.FP64, max_iter=100000)
    dl = torch.tensor(d.l, device=dev)
    D0 = torch.empty_like(dl)
    hjr.solve_device(d.grid, d.dyn, dl, None, D0, **dopt)
    dl2 = torch.tensor(np.minimum(d.l, W.box_sdf(d.grid, (0.6, 0.6), (0.05, 0.05))), device=dev)
    res = {}
    Vs = {}
    for local in (0, 1):
        Vt = torch.empty_like(dl)
        r, st = hjr.solve_device(d.grid, d.dyn, dl2, D0, Vt, local_updates=local, **dopt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r, st = hjr.solve_device(d.grid, d.dyn, dl2, D0, Vt, local_updates=local, **dopt)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / args.steps
        Vs[local] = Vt.cpu().numpy()
        key = "local" if local else "full"
        res[key] = {"seconds": el, "steps": r["iterations"], "node_updates": r["node_updates"], "status": st}
        log(f"di1001 new obstacle {key}: {res[key]}")
    res["bitwise_equal"] = bool(np.array_equal(Vs[0], Vs[1]))
    res["computed_fraction"] = res["local"]["node_updates"] / res["full"]["node_updates"]
    res["speedup"] = res["full"]["seconds"] / res["local"]["seconds"]
    out["di1001^2-upwind-euler-fp64 new-obstacle"] = res
    print(json.dumps({"workload": "local-updates", "scenarios": out}), flush=True)


def bench_control(args):
    """Safe-control queries (Sec. II-B.2, eq. (uOpt)) against the converged 101^3 Dubins value
    function: the WENO5 nodal gradient once, then batches of uniformly drawn states (gradient,
    value and control per state), timed with events on the library's stream."""
    import numpy as np
    import torch

    from paper_1903_07715_amd import hjr
    from paper_1903_07715_amd import workloads as W

    dev = torch.device("cuda:0")
    p = W.dubins_problem(args.n)
    g = p.grid
    lt = torch.tensor(p.l, device=dev)
    Vt = torch.empty_like(lt)
    res, st = hjr.solve_device(g, p.dyn, lt, None, Vt, **hjr.problem_options(p, precision=hjr.FP32_POLISH64))
    log(f"control: value function {res['iterations']}+{res['polish_iterations']} steps, status {st}")
    nq = args.queries
    rng = np.random.default_rng(20190318)
    x = torch.tensor(rng.uniform(g.lo, g.hi, size=(nq, 3)), device=dev)
    table = torch.empty(4 * g.size, dtype=torch.float64, device=dev)
    u = torch.empty(nq, dtype=torch.float64, device=dev)
    pq = torch.empty(3 * nq, dtype=torch.float64, device=dev)
    vq = torch.empty(nq, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            hjr.gradient_device(g, Vt, table, spatial=5, stream=stream)
            hjr.safe_control_device(g, p.dyn, table, x, u, p=pq, v=vq, stream=stream)
        e[0].record(stream)
        for _ in range(args.steps):
            hjr.gradient_device(g, Vt, table, spatial=5, stream=stream)
        e[1].record(stream)
        e[2].record(stream)
        for _ in range(args.steps):
            hjr.safe_control_device(g, p.dyn, table, x, u, p=pq, v=vq, stream=stream)
        e[3].record(stream)
    torch.cuda.synchronize()
    grad_ms = e[0].elapsed_time(e[1]) / args.steps
    q_ms = e[2].elapsed_time(e[3]) / args.steps
    # algorithmic bytes: the table pass reads V and writes 4 values per node (FP64); a query reads
    # its state and the 8 cell-corner records (3 gradient components and V), writes u, p and v
    grad_bytes = g.size * 8 * (1 + 4)
    q_bytes = nq * (3 * 8 + 8 * 4 * 8 + 8 * (1 + 3 + 1))
    log(f"gradient pass {grad_ms * 1e3:.1f} us, {nq} queries {q_ms * 1e3:.1f} us")
    print(json.dumps({"workload": f"safe-control-dubins{args.n}^3-weno5-fp64", "queries": nq,
                      "queries_per_s": nq / (q_ms / 1e3), "query_batch_us": q_ms * 1e3,
                      "gradient_pass_us": grad_ms * 1e3, "unit": "queries/s",
                      "query_algorithmic_gbs": q_bytes / (q_ms / 1e3) / 1e9,
                      "gradient_algorithmic_gbs": grad_bytes / (grad_ms / 1e3) / 1e9,
                      "peak_hbm_gbs": PEAK_HBM_GBS, "steps": args.steps}), flush=True)


def bench_quad10(args):
    """Sec. VI scenario on the 10-D near-hover quadrotor, solved as its x, y (41^4 each) and z
    (201^2) subsystems: value functions for mass 5 and horizontal disturbance 1, then for the
    changed problems (mass 5.25 / disturbance 1.5, and mass 4.8 / disturbance 0.95) cold and
    warm-started from the first, FP32 + FP64 polish, all three subsystems in one batch."""
    import torch

    from paper_1903_07715_amd import hjr
    from paper_1903_07715_amd import workloads as W

    dev = torch.device("cuda:0")
    nxy, nz = 41, 201

    def run(probs, ks):
        ls = [torch.tensor(p.l, device=dev) for p in probs]
        outs = [torch.empty_like(l) for l in ls]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with hjr.Context(0) as ctx:
            ts = [ctx.submit(p.grid, p.dyn, l, k, V, **hjr.problem_options(p, max_iter=50000))
                  for p, l, k, V in zip(probs, ls, ks, outs)]
            ctx.drain()
            res = [ctx.poll(t) for t in ts]
        return outs, res, time.perf_counter() - t0

    m0, d0 = W.QUAD10_SCENARIOS["base"]
    base = W.quad10_problems(m=m0, dbar_xy=d0, n_xy=nxy, n_z=nz)
    run(base, [None] * 3)  # warm-up (tuning, first-touch allocation)
    Vb, rb, tb = run(base, [None] * 3)
    log(f"quad10 base: {[r['iterations'] + r['polish_iterations'] for _, r in rb]} steps, {tb:.3f} s")
    out = {"workload": f"quad10-subsystems-xy{nxy}^4-z{nz}^2-upwind-euler-fp32-polish64",
           "base_steps": [r["iterations"] + r["polish_iterations"] for _, r in rb], "base_seconds": tb}
    for tag in ("heavier", "lighter"):
        m, dxy = W.QUAD10_SCENARIOS[tag]
        new = W.quad10_problems(m=m, dbar_xy=dxy, n_xy=nxy, n_z=nz)
        Vc, rc, tc = run(new, [None] * 3)
        Vw, rw, tw = run(new, Vb)
        err = [float((a - b).abs().max()) for a, b in zip(Vw, Vc)]
        log(f"quad10 {tag}: cold {tc:.3f} s, warm {tw:.3f} s, max |warm - cold| {err}")
        out[tag] = {"mass": m, "dbar_xy": dxy,
                    "cold_steps": [r["iterations"] + r["polish_iterations"] for _, r in rc],
                    "warm_steps": [r["iterations"] + r["polish_iterations"] for _, r in rw],
                    "cold_seconds": tc, "warm_seconds": tw, "speedup": tc / tw,
                    "max_abs_warm_minus_cold": err,
                    "statuses": [s for s, _ in rc] + [s for s, _ in rw]}
    print(json.dumps(out), flush=True)


def bench_hbm(args):
    """The HBM-bound path: FP32 first-order upwind + forward Euler steps of the 6-D quadrotor on
    a 25^6 grid (244 M nodes, about 1 GB per FP32 field, far beyond the 256 MB Infinity Cache).
    One Euler step must read V and l and write V: 12 algorithmic bytes per node.  The stage
    kernel's average duration comes from launch-stamped events over a fixed number of steps."""
    import torch

    from paper_1903_07715_amd import hjr
    from paper_1903_07715_amd import workloads as W

    dev = torch.device("cuda:0")
    p = W.quad6_problem(args.quad_n)
    npts = p.grid.size
    lt = torch.tensor(p.l, device=dev)
    Vt = torch.empty_like(lt)
    steps = 40
    opts = hjr.problem_options(p, precision=hjr.FP32, max_iter=steps)
    log(f"hbm: quad6 {args.quad_n}^6 = {npts} nodes, {steps} Euler steps per solve")
    hjr.solve_device(p.grid, p.dyn, lt, None, Vt, **opts)  # warm-up (tuning, first-touch allocation)
    hjr.solve_device(p.grid, p.dyn, lt, None, Vt, **opts)
    hjr.profile_read(reset=True)
    hjr.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, st = hjr.solve_device(p.grid, p.dyn, lt, None, Vt, **opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hjr.profile_enable(False)
    prof = hjr.profile_read(reset=True)
    avg_s, nwork = working_avg(prof["stage32"])
    gbs = 12.0 * npts / avg_s / 1e9
    log(f"stage kernel {avg_s * 1e6:.1f} us per launch, {gbs:.0f} GB/s algorithmic")
    print(json.dumps({"workload": f"quad6-{args.quad_n}^6-upwind-euler-fp32", "nodes": npts,
                      "steps_per_solve": res["iterations"], "status": st,
                      "grid_point_updates_per_s": args.steps * res["iterations"] * npts / el,
                      "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                   "frac": round(gbs / PEAK_HBM_GBS, 4), "avg_launch_us": round(avg_s * 1e6, 1),
                                   "working_launches": nwork,
                                   "kernel": kernel_name(tuner_config(False, p.dyn.id, 1, npts), False, "Quad6")}}),
          flush=True)


def bench_batch(args):
    """64 seeded mixed instances (double integrator 51^2-201^2, Dubins 41^3-121^3), FP32,
    device-resident, advanced together by the serving context (every stage of every instance
    in the same launches), against the same solves one after another."""
    import torch

    from paper_1903_07715_amd import hjr
    from paper_1903_07715_amd import workloads as W

    dev = torch.device("cuda:0")
    probs = W.batch_problems(64)
    ls = [torch.tensor(p.l, device=dev) for p in probs]
    outs = [torch.empty_like(l) for l in ls]
    opts = [hjr.problem_options(p, precision=hjr.FP32, max_iter=20000) for p in probs]
    npts = sum(p.grid.size for p in probs)
    log(f"batch: {len(probs)} instances, {npts} nodes")
    torch.cuda.synchronize()

    def batched():
        with hjr.Context(0) as ctx:
            ts = [ctx.submit(p.grid, p.dyn, l, None, V, **o) for p, l, V, o in zip(probs, ls, outs, opts)]
            ctx.drain()
            res = [ctx.poll(t) for t in ts]
            stats = ctx.stats()
        return res, stats

    batched()  # warm-up (tuning, first-touch allocation)
    t0 = time.perf_counter()
    res, stats = batched()
    bt = time.perf_counter() - t0
    upd = sum((r["iterations"] + r["polish_iterations"]) * p.grid.size for (_, r), p in zip(res, probs))
    log(f"batched: {bt:.3f} s, {stats['chunks']} chunks, {stats['launches']} launches")
    t0 = time.perf_counter()
    for p, l, V, o in zip(probs, ls, outs, opts):
        hjr.solve_device(p.grid, p.dyn, l, None, V, **o)
    torch.cuda.synchronize()
    st = time.perf_counter() - t0
    log(f"one by one: {st:.3f} s")
    ok = sum(1 for s_, _ in res if s_ == hjr.OK)
    print(json.dumps({"workload": "batch64-di-dubins-upwind-euler-fp32", "instances": len(probs), "nodes": npts,
                      "batched_seconds": bt, "sequential_seconds": st, "batched_solves_per_s": ok / bt,
                      "sequential_solves_per_s": ok / st, "speedup": st / bt,
                      "grid_point_updates_per_s": upd / bt, "converged": ok, "not_converged": len(res) - ok,
                      "statuses": sorted(set(s_ for s_, _ in res)), "launches": stats["launches"],
                      "chunks": stats["chunks"]}), flush=True)


def bench_serve(args):
    """Poisson stream of reachability requests whose parameters change (quadrotor mass and
    disturbance, Dubins and double-integrator control and disturbance bounds, unicycle
    disturbance), through the serving context, warm-started from resident prior solutions vs
    cold, on the same arrival trace."""
    import random

    import torch

    from paper_1903_07715_amd import hjr, serving
    from paper_1903_07715_amd import workloads as W

    dev = torch.device("cuda:0")
    rng = random.Random(W.SEED)
    kinds = {}
    qn = args.quad_n
    quad = W.quad6_problem(qn)
    kinds["quad6"] = (quad, torch.tensor(quad.l, device=dev))
    dub = W.dubins_problem(101, scheme="upwind")  # WENO5 has no steady state for most parameter draws
    kinds["dubins3"] = (dub, torch.tensor(dub.l, device=dev))
    uni = W.unicycle_problem(61)
    uni.spatial, uni.temporal, uni.cfl = 1, 1, 0.8  # converged solves need the monotone scheme here
    kinds["unicycle4"] = (uni, torch.tensor(uni.l, device=dev))
    di = W.di_box_problem(101)
    kinds["di2"] = (di, torch.tensor(di.l, device=dev))

    def make(kind, arrival):
        p, l_t = kinds[kind]
        if kind == "quad6":
            m, db = rng.uniform(1.0, 1.4), rng.uniform(0.2, 0.8)
            dyn, key = W.quad6(m=m, dbar=(db, db, db)), (m, db)
            # the prior dominates when its vertical acceleration interval [T_min/m - g, T_max/m - g]
            # contains the new one and its disturbance is no larger; with T_min > 0 a mass change
            # moves both ends the same way, so only equal masses qualify
            acc = lambda mm: (5.0 / mm - 9.81, 20.0 / mm - 9.81)
            dom = lambda a, b: (acc(a[0])[0] <= acc(b[0])[0] and acc(a[0])[1] >= acc(b[0])[1] and a[1] <= b[1])
        elif kind == "dubins3":
            ub, db = rng.uniform(1.0, 2.0), rng.uniform(0.0, 0.2)
            dyn, key = W.dubins3(1.0, ub, db), (-ub, db)
            dom = lambda a, b: a[0] <= b[0] and a[1] <= b[1]       # more control, less disturbance
        elif kind == "unicycle4":
            # the 4-D configuration's disturbance bound is 0.1; above it (0.105-0.147 measured)
            # the upwind iteration on the bounded 61^4 grid keeps changing by 1e-5-7e-5 per step
            # for 20000 FP64 steps, i.e. has no steady state to converge to
            db = rng.uniform(0.0, 0.1)
            dyn, key = W.unicycle4(1.0, 0.5, db), (db,)
            dom = lambda a, b: a[0] <= b[0]
        else:
            ub, db = rng.uniform(0.5, 2.0), rng.uniform(0.0, 0.2)
            dyn, key = W.double_integrator(ub, 1.0, db), (-ub, db)
            dom = lambda a, b: a[0] <= b[0] and a[1] <= b[1]
        opts = hjr.problem_options(p, precision=hjr.FP32_POLISH64, max_iter=20000, polish_shift=args.polish_shift)
        return serving.Request(kind=kind, grid=p.grid, dyn=dyn, key=key, dominates=dom, l_dev=l_t, opts=opts,
                               arrival=arrival)

    mix = ["quad6"] * 4 + ["dubins3"] * 2 + ["unicycle4"] * 2 + ["di2"] * 2
    # calibration: one cold solve of each kind alone gives the mean service time
    svc = {}
    for kind in kinds:
        r = make(kind, 0.0)
        V = torch.empty_like(r.l_dev)
        t0 = time.perf_counter()
        hjr.solve_device(r.grid, r.dyn, r.l_dev, None, V, **r.opts)
        torch.cuda.synchronize()
        svc[kind] = time.perf_counter() - t0
        log(f"calibration {kind}: {svc[kind]:.3f} s")
    mean_svc = sum(svc[k] for k in mix) / len(mix)
    rate = 0.7 / mean_svc
    log(f"arrival rate {rate:.2f}/s (0.7 x one-at-a-time capacity)")
    rng.seed(W.SEED + 1)
    t = 0.0
    trace = []
    for _ in range(args.requests):
        t += rng.expovariate(rate)
        trace.append((rng.choice(mix), t))
    out = {}

    def per_kind(reqs):
        kk = {}
        for r in reqs:
            d = kk.setdefault(r.kind, {"n": 0, "steps": 0, "latency_s": 0.0, "statuses": set()})
            d["n"] += 1
            d["steps"] += r.result.get("iterations", 0) + r.result.get("polish_iterations", 0)
            d["latency_s"] += r.done - r.arrival
            d["statuses"].add(r.status)
        return {k: {"n": v["n"], "mean_steps": v["steps"] / v["n"], "mean_latency_s": v["latency_s"] / v["n"],
                    "statuses": sorted(v["statuses"])} for k, v in kk.items()}

    def progress(r, k):
        if k % 32 == 0:
            log(f"  {k} requests done")

    # 1) Poisson arrivals at 0.7x the one-at-a-time capacity: latency, warm vs cold
    for warm in (False, True):
        rng.seed(W.SEED + 2)
        reqs = [make(kind, at) for kind, at in trace]
        with hjr.Context(0, args.serve_budget_gb << 30) as ctx:
            srv = serving.WarmStartServer(ctx, warm=warm, keep_outputs=False)
            srv.run(reqs, torch, dev, max_in_flight=args.serve_in_flight, on_done=progress)
            stats = ctx.stats()
        st = serving.latency_stats(reqs)
        st["steps"] = sum(r.result.get("iterations", 0) + r.result.get("polish_iterations", 0) for r in reqs)
        st["statuses"] = sorted(set(r.status for r in reqs))
        st["warm_started"] = sum(1 for r in reqs if r.warm_from is not None)
        st["warm_from_dominating_prior"] = sum(1 for r in reqs if r.exact_warm)
        st["hbm_peak_bytes"] = stats["bytes_peak"]
        st["per_kind"] = per_kind(reqs)
        out["warm" if warm else "cold"] = st
        if warm:
            prior_store = srv.resident
        log(f"poisson {'warm' if warm else 'cold'}: {st}")
    # 2) the same requests all at once (saturation): serving loop warm/cold vs plain cold solves
    sat = {}
    # fresh parameter draws (seed differs from the Poisson pass); the warm pass starts with the
    # solutions the warm Poisson pass left resident, i.e. of other parameter values
    for warm in (False, True):
        rng.seed(W.SEED + 3)
        reqs = [make(kind, 0.0) for kind, _ in trace]
        with hjr.Context(0, args.serve_budget_gb << 30) as ctx:
            srv = serving.WarmStartServer(ctx, warm=warm, keep_outputs=False)
            if warm:
                srv.resident = prior_store
            srv.run(reqs, torch, dev, max_in_flight=args.serve_in_flight, on_done=progress)
        st = serving.latency_stats(reqs)
        sat["warm" if warm else "cold"] = {"solves_per_s": st["solves_per_s"], "seconds": st["seconds"],
                                            "steps": sum(r.result.get("iterations", 0) + r.result.get("polish_iterations", 0) for r in reqs)}
        log(f"burst {'warm' if warm else 'cold'}: {sat['warm' if warm else 'cold']}")
    rng.seed(W.SEED + 3)
    reqs = [make(kind, 0.0) for kind, _ in trace]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        V = torch.empty_like(r.l_dev)
        hjr.solve_device(r.grid, r.dyn, r.l_dev, None, V, **r.opts)
    torch.cuda.synchronize()
    plain = len(reqs) / (time.perf_counter() - t0)
    sat["plain_cold_solves_per_s"] = plain
    log(f"plain cold one at a time: {plain:.2f} solves/s")
    print(json.dumps({"workload": f"serve-quad6-{qn}^6-dubins101^3-unicycle61^4-di101^2", "requests": args.requests,
                      "arrival_rate_per_s": rate, "cold": out["cold"], "warm": out["warm"], "burst": sat,
                      "warm_serving_vs_plain_cold_solves_per_s": sat["warm"]["solves_per_s"] / plain}),
          flush=True)


if __name__ == "__main__":
    main()
