#!/usr/bin/env python3
"""Throughput of the biofilm time step on one MI355X.

Workload: the 3D square tube of 64 x 64 x 128 cells (walls on the sides,
laminar inflow, free outflow) with 5 000 seeded Poisson-disc nodes in a
Gaussian mound on the bottom wall, springs to neighbours within 2.5 um,
density ratio 1.05, viscosity ratio 100, V(2,2) cycles to 1e-10 relative
residual, coarse viscosity scaled by 0.7 (eq:ViscCoarseGrid).  One step is the whole path: momentum right-hand side, viscous and
pressure multigrid solves, projection, interpolation, node move, spring
breakage and forces, spread, coefficient hierarchy.

The metric is multigrid-solve throughput, unknowns solved per second of
solve time (device time from right-hand side ready to converged), summed
over both solves of every timed step; the FP32-refined solver (four FP32
V-cycles per FP64 correction) gives `value`, the plain FP64 solver is
reported beside it.  Step latency percentiles are
wall-clock per step.  The dominant finest-level kernel is timed live with HIP
events on the context's stream and set against the HBM roofline using its
algorithmic bytes per unknown.  The timed steps replay each solver iteration
as a HIP graph, which carries no per-kernel events; the kernel durations come
from as many further steps taken with one launch per kernel (the same kernels
and launch shapes), right after the timed ones.  The CPU baseline times the FP64 oracle on a
bounded sample of the same workload.

With the viscosity made uniform (mu_max = mu_out) the bench also steps the
same workload with the coupled viscous system and with the constant-viscosity
form of eq:NSdis1 (each component solved on its own, one smoothing launch
per colour for all components) and reports both (`constant_viscosity`).

`--workload serving` runs the serving stream instead: independent requests of
mixed grids and contrasts arriving over time, admitted by slot cap and
device-memory budget and stepped together; it prints its own line with the
aggregate solve DOF/s and the p50/p99 step and request latencies.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MG solve DOF/s at 1e-10 rel residual, FP32-refined vs FP64; p50/p99 latency"

# kernel classes of ibb_profile_read and their algorithmic bytes per unknown
# (minimum traffic of one full update or evaluation, in units of the word size)
CLASS_NAMES = {0: "smooth_u_f64", 1: "smooth_p_f64", 2: "smooth_u_f32", 3: "smooth_p_f32", 4: "resid_u_f64",
               5: "resid_p_f64"}
KERNEL_SYMBOLS = {0: "k_smooth_u<double>", 1: "k_smooth_p<double>", 2: "k_smooth_u<float>", 3: "k_smooth_p<float>",
                  4: "k_resid_u<double>", 5: "k_resid_p<double>"}


def words_per_unknown(cls, D, decoupled=False):
    if decoupled and cls in (0, 2, 4):   # u_a read+write, b, rho
        return 4
    if cls in (0, 2, 4):   # u_a read+write (residual: read + r write), b, rho, mu_c, D-1 mu_e, D-1 u_b
        return 5 + 2 * (D - 1)
    return 2 + 1 + D       # p read+write (residual: read + r write), b, D beta


def word_size(cls):
    return 4 if cls in (2, 3) else 8


def source_digest():
    h = hashlib.sha256()
    for name in sorted(os.listdir(os.path.join(ROOT, "paper_1302_3663_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1302_3663_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(cls, workload):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{CLASS_NAMES[cls]}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    m_val = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_val or m_sha.group(1) != source_digest():
        return None
    return float(m_val.group(1))


def percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q)) if v else None


def run_mode(case, precision, inner, steps, warmup, log, krylov=0, prof_steps=0):
    """Warm up, then time `steps` steps as the library runs them (each
    solver iteration one graph replay).  Then, with kernel timing on (one
    launch per kernel, dispatch-recorded HIP events on the context's stream),
    take `prof_steps` more steps for the per-kernel durations."""
    import torch

    from paper_1302_3663_amd import ibmg
    if krylov:
        case = dict(case, params=dict(case["params"], krylov_restart=krylov))
    ctx = ibmg.from_case(case, precision=precision, inner_cycles=inner)
    for _ in range(warmup):
        ctx.projection_step()
        ctx.lagrangian_update()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms, dof, solve_ms, cyc_u, cyc_p, vcyc, relres = [], 0, 0.0, [], [], [], []
    for k in range(steps):
        ts = time.perf_counter()
        s = ctx.projection_step()
        ctx.lagrangian_update()
        step_ms.append((time.perf_counter() - ts) * 1e3)
        dof += s["dof_u"] + s["dof_p"]
        solve_ms += s["t_u_ms"] + s["t_p_ms"]
        cyc_u.append(s["cycles_u"])
        cyc_p.append(s["cycles_p"])
        vcyc.append(s["vcycles_u"] + s["vcycles_p"])
        relres.append(max(s["relres_u"], s["relres_p"]))
        log(f"  step {k}: {step_ms[-1]:.2f} ms, cycles u {s['cycles_u']} p {s['cycles_p']}, "
            f"solve {s['t_u_ms'] + s['t_p_ms']:.2f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = {}
    if prof_steps > 0:
        ctx.profile_enable(True)
        for _ in range(prof_steps):
            ctx.projection_step()
            ctx.lagrangian_update()
        torch.cuda.synchronize()
        prof = {cls: ctx.profile_read(cls) for cls in CLASS_NAMES}
        ctx.profile_enable(False)
    ctx.close()
    return dict(dof_per_s=dof / (solve_ms / 1e3), wall_s=wall, ms_per_step=wall * 1e3 / steps, solve_ms=solve_ms,
                dof_total=dof, step_ms=step_ms, cycles_u=cyc_u, cycles_p=cyc_p, vcycles=vcyc,
                max_relres=max(relres), prof=prof)


def cpu_baseline(case, log):
    """The FP64 oracle on one viscous and one pressure solve of the first step."""
    import numpy as np

    import oracle as O
    p = case["params"]
    X = case["X"]
    F, _, _ = O.springs(p, X, case["ij"], case["rest"], case["K"], np.ones(case["ij"].shape[1], np.uint8),
                        do_break=False)
    f = O.spread_vec(p, p["omega"], X, F)
    rho, mc, me = O.density(p, X), O.viscosity_cells(p, X), O.viscosity_edges(p, X)
    H = O.Hierarchy(p, rho, mc, me)
    b = O.momentum_rhs(p, case["u0"], rho, mc, me, f)
    t0 = time.perf_counter()
    ut, su = H.solve(True, b, case["u0"])
    t1 = time.perf_counter()
    bp = O.pressure_rhs(p, ut)
    t2 = time.perf_counter()
    _, sp = H.solve(False, bp, case["p0"])
    t3 = time.perf_counter()
    dof = H.nunk[0][0] + H.nunk[0][1]
    secs = (t1 - t0) + (t3 - t2)
    log(f"  oracle: viscous {t1 - t0:.1f} s ({su['cycles']} cycles), pressure {t3 - t2:.1f} s ({sp['cycles']} cycles)")
    return dict(value=dof / secs, unit="DOF/s", cores=1, kind="oracle",
                sample="one viscous and one pressure solve (FP64, V(2,2) to 1e-10) of the first step of the "
                       f"same workload, {secs:.1f} s single-threaded")


SERVING_METRIC = "serving: aggregate MG solve DOF/s and p50/p99 step latency, mixed request stream"


def run_serving(args, log):
    """The serving stream: args.requests requests (synth.serving_request)
    arriving with exponential gaps at args.rate per second, admitted by slot
    cap and device-memory budget, stepped together (serve.Server)."""
    import torch

    from paper_1302_3663_amd import _lib as L
    from paper_1302_3663_amd import serve, synth
    log(f"serving: generating {args.requests} requests")
    cases = [synth.serving_request(j) for j in range(args.requests)]
    arrivals = serve.poisson_arrivals(args.requests, args.rate, seed=4)
    srv = serve.Server(budget_bytes=int(args.budget_gb * (1 << 30)), max_slots=args.slots,
                       precision=L.IBB_FP32_REFINED, inner_cycles=args.inner, krylov=args.krylov,
                       krylov_ratio=args.krylov_ratio)
    # warmup: a few requests through the same loop (loads the code objects)
    warm = [serve.Request(-1 - j, 0.0, cases[j], 1) for j in range(min(args.warmup, len(cases)))]
    if warm:
        srv.run(warm)
    reqs = [serve.Request(j, a, c, c["steps"]) for j, (a, c) in enumerate(zip(arrivals, cases))]
    k = [0]

    def tick_log(m):
        k[0] += 1
        if k[0] % 10 == 0:
            log(m)
    torch.cuda.synchronize()
    s = srv.run(reqs, log=tick_log)
    sizes = {}
    for c in cases:
        key = "x".join(str(v) for v in c["size"])
        sizes[key] = sizes.get(key, 0) + 1
    steps = sum(r.done for r in reqs)
    return {
        "metric": SERVING_METRIC,
        "value": round(s["solve_dof_per_s"], 1),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": len(warm),
        "ms_per_step": round(1e3 * s["busy_s"] / max(s["ticks"], 1), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-inner/f64-outer",
        "data": "synthetic",
        "config": {"workload": "serving", "requests": args.requests, "rate_per_s": args.rate,
                   "steps_per_request": cases[0]["steps"], "slots": args.slots, "budget_gb": args.budget_gb,
                   "sizes": sizes, "inner_cycles": args.inner,
                   "gcr": {"restart": args.krylov, "from_viscosity_ratio": args.krylov_ratio} if args.krylov else None},
        "p50_step_ms": round(s["p50_step_ms"], 3),
        "p99_step_ms": round(s["p99_step_ms"], 3),
        "p50_request_s": round(s["p50_request_s"], 3),
        "p99_request_s": round(s["p99_request_s"], 3),
        "p50_wait_s": round(s["p50_wait_s"], 3),
        "p99_wait_s": round(s["p99_wait_s"], 3),
        "wall_s": round(s["wall_s"], 3),
        "ticks": s["ticks"],
        "mean_resident": round(s["mean_resident"], 2),
        "peak_resident": s["peak_resident"],
        "peak_bytes": s["peak_bytes"],
        "busy_dof_per_s": round(s["busy_dof_per_s"], 1),
        "failed_steps": s["failed_steps"],
        "roofline": None,
        "cpu_baseline": None,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--inner", type=int, default=None,
                    help="FP32 V-cycles per FP64 outer iteration (default 4; 2 for the serving stream, whose small "
                         "grids converge in a few cycles, so that larger counts overshoot)")
    ap.add_argument("--modes", default="both", choices=["both", "fp64", "refined"])
    ap.add_argument("--workload", default="tube3d_64x64x128",
                    help="a synth.WORKLOADS entry, or 'serving' for the mixed request stream")
    ap.add_argument("--requests", type=int, default=256, help="serving: number of requests")
    ap.add_argument("--rate", type=float, default=40.0, help="serving: arrivals per second")
    ap.add_argument("--slots", type=int, default=32, help="serving: resident request cap")
    ap.add_argument("--budget-gb", type=float, default=32.0, help="serving: device-memory budget")
    ap.add_argument("--krylov-ratio", type=float, default=100.0,
                    help="serving: GCR for requests with at least this viscosity ratio (with --krylov > 0)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--krylov", type=int, default=8, metavar="M",
                    help="also time the GCR(M)-accelerated solver in each mode (0: skip)")
    ap.add_argument("--gcr-inner", type=int, default=2,
                    help="FP32 V-cycles per preconditioner application of refined GCR (cheaper applications "
                         "suit GCR: 2 beat 4 on both tubes)")
    ap.add_argument("--const-visc", type=int, default=1, choices=[0, 1],
                    help="also step the workload at uniform viscosity, coupled and constant-viscosity form")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.inner is None:
        args.inner = 2 if args.workload == "serving" else 4
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported by this build", file=sys.stderr)
        sys.exit(2)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    import numpy as np
    import torch

    import paper_1302_3663_amd as pkg
    from paper_1302_3663_amd import synth
    pkg.load()   # raises when the HIP library is missing: there is no fallback
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "serving":
        print(json.dumps(run_serving(args, log)), flush=True)
        return
    log(f"workload {args.workload}: generating inputs")
    case = synth.WORKLOADS[args.workload]()
    p = case["params"]
    modes = {"both": ["fp64", "refined"], "fp64": ["fp64"], "refined": ["refined"]}[args.modes]
    res = {}
    for m in modes:
        log(f"mode {m}: {args.warmup} warmup + {args.steps} timed steps")
        res[m] = run_mode(case, pkg.IBB_FP32_REFINED if m == "refined" else pkg.IBB_FP64, args.inner, args.steps,
                          args.warmup, log, prof_steps=args.steps)
    gcr = {}
    if args.krylov > 0:
        for m in modes:
            log(f"mode {m} with GCR({args.krylov}): {args.warmup} warmup + {args.steps} timed steps")
            gcr[m] = run_mode(case, pkg.IBB_FP32_REFINED if m == "refined" else pkg.IBB_FP64, args.gcr_inner,
                              args.steps, args.warmup, log, krylov=args.krylov)
    const = {}
    if args.const_visc:
        for dec in (0, 1):
            # uniform viscosity: restricted coefficients are exact, no coarse scaling
            cp = dict(case["params"], mu_max=case["params"]["mu_out"], decoupled=dec, gamma=[1.0] * 16)
            log(f"uniform viscosity, {'constant-viscosity form' if dec else 'coupled form'}: "
                f"{args.warmup} warmup + {args.steps} timed steps")
            const[dec] = run_mode(dict(case, params=cp), pkg.IBB_FP32_REFINED if "refined" in modes else pkg.IBB_FP64,
                                  args.inner, args.steps, args.warmup, log, prof_steps=args.steps)
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 copies of {args.calibrate_copy} MiB")
    head = res["refined"] if "refined" in res else res["fp64"]
    head_mode = "refined" if "refined" in res else "fp64"
    # roofline of the dominant finest-level kernel of the headline mode
    D = p["dim"]
    dom = max(head["prof"], key=lambda c: head["prof"][c]["total_ms"])
    pr = head["prof"][dom]
    bpu = words_per_unknown(dom, D) * word_size(dom)
    per_launch_bytes = bpu * pr["units"] / max(pr["launches"], 1)
    avg_ms = pr["total_ms"] / max(pr["launches"], 1)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    traffic = committed_traffic(dom, args.workload)
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=KERNEL_SYMBOLS[dom],
                avg_launch_us=round(avg_ms * 1e3, 2), launches=pr["launches"],
                algorithmic_bytes_per_launch=int(per_launch_bytes), bytes_per_unknown=bpu)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle")
        cpu = cpu_baseline(case, log)
    all_steps = head["step_ms"]
    out = {
        "metric": METRIC,
        "value": round(head["dof_per_s"], 1),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-inner/f64-outer" if head_mode == "refined" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": p["n"][:p["dim"]], "nodes": int(case["X"].shape[1]),
                   "springs": int(case["ij"].shape[1]), "viscosity_ratio": p["mu_max"] / p["mu_out"],
                   "density_ratio": (p["rho0"] + p["rho_b"]) / p["rho0"], "rtol": p["rtol"],
                   "nu": [p["nu1"], p["nu2"]], "gamma_2h": p["gamma"][1], "precision": head_mode,
                   "inner_cycles": args.inner if head_mode == "refined" else None},
        "p50_step_ms": round(percentile(all_steps, 50), 3),
        "p99_step_ms": round(percentile(all_steps, 99), 3),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    for m in res:
        r = res[m]
        out[m] = dict(dof_per_s=round(r["dof_per_s"], 1), ms_per_step=round(r["ms_per_step"], 3),
                      solve_ms_per_step=round(r["solve_ms"] / args.steps, 3),
                      mean_cycles_u=float(np.mean(r["cycles_u"])), mean_cycles_p=float(np.mean(r["cycles_p"])),
                      mean_vcycles=float(np.mean(r["vcycles"])), max_relres=r["max_relres"],
                      p50_step_ms=round(percentile(r["step_ms"], 50), 3),
                      p99_step_ms=round(percentile(r["step_ms"], 99), 3),
                      kernels={CLASS_NAMES[c]: dict(launches=v["launches"], avg_us=round(
                          1e3 * v["total_ms"] / max(v["launches"], 1), 2), total_ms=round(v["total_ms"], 3))
                          for c, v in r["prof"].items() if v["launches"]})
    if "fp64" in res and "refined" in res:
        out["refined_over_fp64"] = round(res["refined"]["dof_per_s"] / res["fp64"]["dof_per_s"], 3)
    if gcr:
        out["gcr"] = {"restart": args.krylov, "inner_cycles": args.gcr_inner}
        for m, r in gcr.items():
            out["gcr"][m] = dict(dof_per_s=round(r["dof_per_s"], 1), ms_per_step=round(r["ms_per_step"], 3),
                                 solve_ms_per_step=round(r["solve_ms"] / args.steps, 3),
                                 mean_cycles_u=float(np.mean(r["cycles_u"])),
                                 mean_cycles_p=float(np.mean(r["cycles_p"])), max_relres=r["max_relres"],
                                 p50_step_ms=round(percentile(r["step_ms"], 50), 3),
                                 p99_step_ms=round(percentile(r["step_ms"], 99), 3),
                                 speedup_vs_plain=round(r["dof_per_s"] / res[m]["dof_per_s"], 3))
    if const:
        sm = 2 if "refined" in modes else 0
        cv = {"viscosity_ratio": 1.0, "precision": head_mode}
        for dec, key in ((0, "coupled"), (1, "decoupled")):
            r = const[dec]
            pr = r["prof"][sm]
            avg_ms = pr["total_ms"] / max(pr["launches"], 1)
            bpl = words_per_unknown(sm, D, bool(dec)) * word_size(sm) * pr["units"] / max(pr["launches"], 1)
            gbs = bpl / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
            cv[key] = dict(dof_per_s=round(r["dof_per_s"], 1), ms_per_step=round(r["ms_per_step"], 3),
                           solve_ms_per_step=round(r["solve_ms"] / args.steps, 3),
                           mean_cycles_u=float(np.mean(r["cycles_u"])), mean_cycles_p=float(np.mean(r["cycles_p"])),
                           max_relres=r["max_relres"],
                           smoother=dict(kernel="k_smooth_u_dec" if dec else KERNEL_SYMBOLS[sm],
                                         launches=pr["launches"], avg_launch_us=round(avg_ms * 1e3, 2),
                                         algorithmic_bytes_per_launch=int(bpl), achieved_gbs=round(gbs, 1),
                                         frac=round(gbs / HBM_PEAK_GBS, 4)))
        cv["decoupled_over_coupled"] = round(const[1]["dof_per_s"] / const[0]["dof_per_s"], 3)
        out["constant_viscosity"] = cv
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
