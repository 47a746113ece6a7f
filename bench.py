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

# launch sites of ibb_profile_read (class = site + 32 x level): kernel symbol,
# word size, and algorithmic words moved per unit (per unknown updated or
# evaluated; a restriction per coarse unknown, the coarse cycle per unknown
# of its start level) -- the minimum traffic of one pass
SITES = {
    0: ("k_smooth_u<double>", 8), 1: ("k_smooth_p<double>", 8), 2: ("k_smooth_u<float>", 4),
    3: ("k_smooth_p<float>", 4), 4: ("k_resid_u<double>", 8), 5: ("k_resid_p<double>", 8),
    6: ("k_resid_u<float>", 4), 7: ("k_resid_p<float>", 4), 8: ("k_restrict<double>", 8),
    9: ("k_restrict<float>", 4), 10: ("k_prolong_add<double>", 8), 11: ("k_prolong_add<float>", 4),
    12: ("k_coarse_vcycle<double, D, 1>", 8), 13: ("k_coarse_vcycle<double, D, 0>", 8),
    14: ("k_coarse_vcycle<float, D, 1>", 4), 15: ("k_coarse_vcycle<float, D, 0>", 4),
    16: ("k_dense_apply", 8), 17: ("outer-loop passes (norms, casts, clears, corrections)", 8),
    18: ("GCR vector passes", 8), 19: ("k_smooth_u_dec<double>", 8), 20: ("k_smooth_u_dec<float>", 4),
    21: ("one-launch sweep (k_smooth_rb, k_smooth_zm)<double>", 8),
    22: ("one-launch sweep (k_smooth_rb, k_smooth_zm)<float>", 4),
    23: ("k_spread_face", 8), 24: ("k_spread_visc", 8), 25: ("k_interp", 8), 26: ("k_spring_force", 8),
    27: ("k_gal_build", 8), 28: ("k_gal_smooth<double>", 8), 29: ("k_gal_smooth<float>", 4),
    30: ("k_gal_resid<double>", 8), 31: ("k_gal_resid<float>", 4),
}
VISCOUS_SITES = {0, 2, 4, 6, 12, 14, 21, 22, 27, 28, 29, 30, 31}
PRESSURE_SITES = {1, 3, 5, 7, 13, 15}


def words_per_unit(site, D, decoupled=False):
    """algorithmic words per unit of a launch site (see SITES)"""
    if site in (19, 20) or (decoupled and site in (0, 2, 4, 6)):
        return 4                                   # u_a read+write, b, rho
    if site in (0, 2, 4, 6, 21, 22):               # u_a read+write (residual: read + r), b, rho, mu_c,
        return 5 + 2 * (D - 1)                     # D-1 mu_e, D-1 other components
    if site in (1, 3, 5, 7):
        return 2 + 1 + D                           # p read+write, b, D beta
    if site in (8, 9):
        return 2 ** D + 2                          # fine residual, coarse b written, coarse x cleared
    if site in (10, 11):
        return 2 + 2.0 ** -D                       # fine x read+write, coarse x
    if site in (12, 13, 14, 15):
        return 6                                   # start level x read+write, b, its coefficients
    if site == 23:
        return 2                                   # per lattice point: f and rho written (gather)
    if site == 24:
        return 1                                   # per lattice point: mu written
    if site == 25:
        return 4 ** D + 1                          # per node and component: 4^D face values, U written
    if site == 26:
        return 3 * D + 20 * (D + 3)                # per node: X, F; about 20 springs: partner X, rest, K, ids
    gal = 235 if D == 3 else 31                    # Galerkin row: stencil-box entries
    if site == 27:
        return gal                                 # per coarse unknown: its row written
    if site in (28, 29):
        return gal + 4                             # row, b, x written; the other colour copied (read + write)
    if site in (30, 31):
        return gal + 2                             # row, b, r written (x reads hit the caches)
    return 3


def site_name(site, level, D):
    return SITES[site][0].replace("D,", f"{D},") + f" (level {level})"


def source_digest():
    h = hashlib.sha256()
    for name in sorted(os.listdir(os.path.join(ROOT, "paper_1302_3663_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1302_3663_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(site, level, workload):
    """HBM bytes per launch from the committed counter summary of this launch
    site and level, if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_site{site}_level{level}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    m_val = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_val or m_sha.group(1) != source_digest():
        return None
    return float(m_val.group(1))


def site_table(prof, D, steps, decoupled=False):
    """Rows per launch site and level, largest device time first: launches,
    device ms per step, average launch, algorithmic bytes per launch, the
    bandwidth those bytes imply, and the share of all timed kernels of a step
    (the solves and the Lagrangian update)."""
    total = sum(v["total_ms"] for v in prof.values()) or 1.0
    rows = []
    for cls, v in prof.items():
        site, level = cls % 32, cls // 32
        bpl = words_per_unit(site, D, decoupled) * SITES[site][1] * v["units"] / v["launches"]
        avg = v["total_ms"] / v["launches"]
        rows.append(dict(site=site, level=level, kernel=site_name(site, level, D), launches=v["launches"],
                         ms_per_step=v["total_ms"] / steps, avg_us=avg * 1e3, bytes_per_launch=bpl,
                         gbs=bpl / (avg * 1e-3) / 1e9 if avg > 0 else 0.0, share=v["total_ms"] / total))
    rows.sort(key=lambda r: -r["ms_per_step"])
    return rows, total


def unknown_extents(p, level, vmask):
    """extent of the unknowns of a lattice along each axis on a level"""
    ext = []
    for d in range(p["dim"]):
        n = p["n"][d] >> level
        if not (vmask >> d) & 1:
            ext.append(n)
        else:
            ext.append({0: n, 1: n - 1, 2: n}[p["axis_bc"][d]])
    return ext + [1] * (3 - p["dim"])


def site_launches(p, site, level):
    """(kernel symbol, grid size in work-items or None for any) of the
    launches of a smoother or coarse-cycle site, as rocprofv3 names them"""
    D = p["dim"]
    T = "float" if SITES[site][1] == 4 else "double"
    if site in (12, 13, 14, 15):
        return [(f"k_coarse_vcycle<{T}, {D}, {1 if site in (12, 14) else 0}>", None)]
    out = []
    if site in (21, 22):
        # one launch per sweep: the z-marching velocity sweep (3D; tiles of
        # 64 x 8 points, runs of planes as the library picks them) or the
        # tiled one (8 x 8 x (8 in FP32, 4 in FP64) tiles; 16 x 16 in 2D),
        # whichever the run used
        for a in range(D):
            e = unknown_extents(p, level, 1 << a)
            if D == 3:
                tiles = -(-e[0] // 64) * -(-e[1] // 8)
                runs = max(1, min(-(-8192 // tiles), e[2] // 4))
                cz = -(-e[2] // runs)
                out.append((f"k_smooth_zm<{T}, {a}>", 256 * tiles * -(-e[2] // cz)))
            t = (8, 8, 8 if T == "float" else 4) if D == 3 else (16, 16, 1)
            nt = -(-e[0] // t[0]) * -(-e[1] // t[1]) * (-(-e[2] // t[2]) if D == 3 else 1)
            out.append((f"k_smooth_rb<{T}, {D}, 1, {a}>", 256 * nt))
        return out
    if site in (0, 2):
        comps = [(f"k_smooth_u<{T}, {D}, {a}>", 1 << a) for a in range(D)]
    elif site in (1, 3):
        comps = [(f"k_smooth_p<{T}, {D}>", 0)]
    else:
        return []
    for sym, vmask in comps:
        e = unknown_extents(p, level, vmask)
        n = ((e[0] + 1) // 2) * e[1] * e[2]
        out.append((sym, 256 * ((n + 255) // 256)))
    return out


def rocprof_average(p, site, level, workload):
    """Average launch duration (us) of a launch site from the committed
    rocprofv3 summary of this workload (rows per kernel symbol and grid
    size), when that summary was taken on the current kernel sources; else
    None."""
    path = os.path.join(ROOT, "profiles", f"launch_sites_{workload}.md")
    want = site_launches(p, site, level)
    if not os.path.exists(path) or not want:
        return None
    text = open(path).read()
    m_sha = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    if not m_sha or m_sha.group(1) != source_digest():
        return None
    calls, total = 0, 0.0
    for line in text.splitlines():
        cells = [c.strip().strip("`") for c in line.split("|")]
        if len(cells) < 6:
            continue
        for sym, grid in want:
            if cells[1] == sym and (grid is None or cells[2] == str(grid)):
                try:
                    c, avg = int(cells[3]), float(cells[4])
                except ValueError:
                    continue
                calls += c
                total += c * avg
    return round(total / calls, 3) if calls else None


def summarize_trace(csv_path, out_path, workload, command):
    """rocprofv3 kernel-trace CSV -> markdown rows per kernel symbol and grid
    size (calls, average and total device time), with the command that took
    the trace and the digest of the kernel sources it ran."""
    import csv
    rows = {}
    spans = []
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            name = r.get("Kernel_Name", "")
            m = re.search(r"(k_\w+)(<[^()]*>)?", name)
            sym = (m.group(1) + (m.group(2) or "")) if m else name.split("(")[0]
            if "Grid_Size_X" in r:
                grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            else:
                grid = int(r.get("Grid_Size", 0))
            t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            us = (t1 - t0) / 1e3
            spans.append((t0, t1, sym))
            e = rows.setdefault((sym, grid), [0, 0.0])
            e[0] += 1
            e[1] += us
    total_ms = sum(v[1] for v in rows.values()) / 1e3
    lines = [f"# Launch sites: {workload}", "", "Command (run from /tmp with TMPDIR=/tmp on one MI355X):", "", "```",
             command, "```", "", f"Kernels by symbol and grid size (work-items), largest total first; all kernels "
             f"{total_ms:.1f} ms.", "", "| kernel | grid | calls | avg us | total ms |", "|---|---:|---:|---:|---:|"]
    for (sym, grid), (n, us) in sorted(rows.items(), key=lambda kv: -kv[1][1])[:60]:
        lines.append(f"| `{sym}` | {grid} | {n} | {us / n:.3f} | {us / 1e3:.3f} |")
    # idle device time: from the end of the kernels so far to the next start;
    # and, after each k_reduce_final (a solver iteration's last kernel), the
    # time to the next kernel that is not the runtime's copy bringing the
    # norm to the host: the host's round trip between two iterations
    spans.sort()
    gaps, turn, copies = [], [], 0
    end = spans[0][1] if spans else 0
    for i, (t0, t1, sym) in enumerate(spans[:-1]):
        end = max(end, t1)
        gaps.append(max(0, spans[i + 1][0] - end) / 1e3)
        if sym == "k_reduce_final":
            j = i + 1
            while j < len(spans) and "copyBuffer" in spans[j][2]:
                j += 1
            if j < len(spans):
                copies += j > i + 1
                turn.append(max(0, spans[j][0] - t1) / 1e3)
    if spans:
        span_ms = (max(t1 for _, t1, _ in spans) - spans[0][0]) / 1e6
        idle = sum(gaps) / 1e3
        med = lambda v: sorted(v)[len(v) // 2] if v else float("nan")
        lines += ["", "Idle device time between kernels over the whole run (from the end of the kernels so far to the "
                  f"next start): {idle:.1f} ms of a {span_ms:.1f} ms span ({100 * idle / span_ms:.1f}%), median gap "
                  f"{med(gaps):.2f} us.  From the end of a `k_reduce_final` (the last kernel of a solver iteration) "
                  "to the next kernel that is not the runtime's copy of the norm to the host (the host reads the "
                  f"norm, then replays the next iteration or ends the solve): {len(turn)} times ({copies} with the "
                  f"copy between), median {med(turn):.2f} us, {sum(turn) / 1e3:.1f} ms in all."]
    lines += ["", f"source_digest: {source_digest()}", ""]
    with open(out_path, "w") as f:
        f.write("\n".join(lines))


def summarize_counters(pmc_dir, workload, site, level, copy_mib, commands, out_path):
    """Four rocprofv3 --pmc runs of the same command (subdirectories fetch:
    FETCH_SIZE; write: WRITE_SIZE; rdreq: TCC_EA0_RDREQ_128B/64B/32B_sum;
    wrreq: TCC_EA0_WRREQ_sum, TCC_EA0_WRREQ_64B_sum) -> the L2-to-fabric
    bytes per launch of one launch site, from the request counts by size,
    with FETCH_SIZE and WRITE_SIZE scaled by what they read for the
    command's plain device copy of copy_mib MiB beside them."""
    import csv
    import collections
    from paper_1302_3663_amd import synth
    p = synth.WORKLOADS[workload]()["params"]
    want = site_launches(p, site, level)

    def load(sub):
        per = collections.defaultdict(lambda: collections.defaultdict(float))
        info = {}
        with open(os.path.join(pmc_dir, sub, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                d = int(r["Dispatch_Id"])
                per[d][r["Counter_Name"]] += float(r["Counter_Value"])
                m = re.search(r"(k_\w+)(<[^()]*>)?", r["Kernel_Name"])
                sym = (m.group(1) + (m.group(2) or "")) if m else r["Kernel_Name"].split("(")[0]
                info[d] = (sym, int(r["Grid_Size"]), "copyBuffer" in r["Kernel_Name"])
        return per, info

    def select(per, info, copy):
        rows = []
        # the calibration copy: the copies of the largest grid (torch's
        # uploads are copies too, of other sizes)
        big = max((g for _, g, c in info.values() if c), default=-1)
        for d, cs in per.items():
            sym, grid, is_copy = info[d]
            if copy and is_copy and grid == big:
                rows.append(cs)
            elif not copy and any(sym == w and (g is None or grid == g) for w, g in want):
                rows.append(cs)
        return rows

    def mean(rows, expr):
        return sum(expr(r) for r in rows) / len(rows) if rows else float("nan")
    runs = {k: load(k) for k in ("fetch", "write", "rdreq", "wrreq")}
    rd = lambda r: 128 * r.get("TCC_EA0_RDREQ_128B_sum", 0) + 64 * r.get("TCC_EA0_RDREQ_64B_sum", 0) + \
        32 * r.get("TCC_EA0_RDREQ_32B_sum", 0)
    wr = lambda r: 64 * r.get("TCC_EA0_WRREQ_64B_sum", 0) + \
        32 * (r.get("TCC_EA0_WRREQ_sum", 0) - r.get("TCC_EA0_WRREQ_64B_sum", 0))
    copy_bytes = copy_mib * (1 << 20)
    k_rd = select(*runs["rdreq"], copy=False)
    k_wr = select(*runs["wrreq"], copy=False)
    c_rd = select(*runs["rdreq"], copy=True)
    c_wr = select(*runs["wrreq"], copy=True)
    k_f = select(*runs["fetch"], copy=False)
    k_w = select(*runs["write"], copy=False)
    c_f = select(*runs["fetch"], copy=True)
    c_w = select(*runs["write"], copy=True)
    rd_scale = copy_bytes / mean(c_rd, rd)
    wr_scale = copy_bytes / mean(c_wr, wr)
    read_b, write_b = mean(k_rd, rd) * rd_scale, mean(k_wr, wr) * wr_scale
    f_scale = copy_bytes / (1024 * mean(c_f, lambda r: r["FETCH_SIZE"]))
    w_scale = copy_bytes / (1024 * mean(c_w, lambda r: r["WRITE_SIZE"]))
    fetch_b = 1024 * mean(k_f, lambda r: r["FETCH_SIZE"]) * f_scale
    wsize_b = 1024 * mean(k_w, lambda r: r["WRITE_SIZE"]) * w_scale
    D = p["dim"]
    units = {0: None}
    kernel = site_name(site, level, D)
    lines = [f"# L2-to-fabric traffic: {kernel}, {workload}", "",
             "Four counter runs of the same command, one counter group each (run from /tmp with TMPDIR=/tmp on "
             "one MI355X, each under `timeout -s KILL 150`):", "", "```"] + commands + ["```", "",
             f"The command copies a {copy_mib} MiB device buffer 5 times beside the solver "
             "(`__amd_rocclr_copyBuffer`, known bytes read and written).", "",
             "Every figure is the counter's value times the factor that makes it read the copy's size.", "",
             "| counters | the copy reads (unscaled) | factor | per launch of the site |", "|---|---:|---:|---:|",
             f"| FETCH_SIZE | {mean(c_f, lambda r: r['FETCH_SIZE']) / 1024:.1f} MiB | {f_scale:.4f} | "
             f"{fetch_b / 1e6:.3f} MB |",
             f"| WRITE_SIZE | {mean(c_w, lambda r: r['WRITE_SIZE']) / 1024:.1f} MiB | {w_scale:.4f} | "
             f"{wsize_b / 1e6:.3f} MB |",
             f"| read requests by size (128 B x RDREQ_128B + 64 B x RDREQ_64B + 32 B x RDREQ_32B) | "
             f"{mean(c_rd, rd) / 2**20:.1f} MiB | {rd_scale:.4f} | {read_b / 1e6:.3f} MB |",
             f"| write requests by size (64 B x WRREQ_64B + 32 B x the rest) | {mean(c_wr, wr) / 2**20:.1f} MiB | "
             f"{wr_scale:.4f} | {write_b / 1e6:.3f} MB |", "",
             f"Launches matched: {len(k_rd)} (symbols and grid sizes: "
             + ", ".join(f"`{w}` {g if g is not None else 'any'}" for w, g in want) + ").", "",
             "The derived FETCH_SIZE counts 128-byte reads through TCC_BUBBLE, which reads 0 on this chip, so it "
             "counts a 128-byte read as 64 bytes; its factor (near 2 when the reads are whole lines) restores the "
             "size.  The request counts by size read the copy's own size in some runs and less in others, so they "
             "are scaled the same way; the two readings agree after scaling.  Both count the L2's traffic to the "
             "fabric, which the 256 MB last-level cache serves in part.  The traffic figure is scaled FETCH_SIZE "
             "plus scaled WRITE_SIZE.", "",
             f"source_digest: {source_digest()}", f"hbm_bytes_per_launch: {fetch_b + wsize_b:.0f}", ""]
    with open(out_path, "w") as f:
        f.write("\n".join(lines))


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
        prof = {}
        for cls in range(512):
            r = ctx.profile_read(cls)
            if r["launches"]:
                prof[cls] = r
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
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return dict(value=dof / secs, unit="DOF/s", cores=1, kind="oracle", cpu_model=model,
                host_cpu_count=os.cpu_count(),
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
    srv = serve.Server(budget_bytes=int(args.budget_gb * (1 << 30)), max_slots=args.slots or None,
                       precision=L.IBB_FP32_REFINED, inner_cycles=args.inner, krylov=args.krylov,
                       krylov_ratio=args.krylov_ratio, max_active=args.active or None)
    # warmup: the stream's first requests, one step each, arriving at once,
    # through the same server: loads the code objects and leaves a pool of
    # slots (at most the concurrency cap) that the timed stream reuses
    nwarm = min(max(args.warmup, args.active or 0), len(cases))
    warm = [serve.Request(-1 - j, 0.0, cases[j], 1) for j in range(nwarm)]
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
    srv.close()
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
                   "steps_per_request": cases[0]["steps"], "slot_cap": args.slots or None,
                   "active_cap": args.active or None, "budget_gb": args.budget_gb, "warm_requests": nwarm,
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
        "group_build_s": round(s["group_build_s"], 3),
        "wall_outside_ticks_s": round(s["wall_outside_ticks_s"], 3),
        "slots": s["slots"],
        "group_builds": s["group_builds"],
        "slots_given_back": s["slots_given_back"],
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
    ap.add_argument("--slots", type=int, default=0, help="serving: cap on the pool of slots (0: the budget binds)")
    ap.add_argument("--active", type=int, default=32,
                    help="serving: cap on the requests stepped together (0: none)")
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
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="also run the serving stream with this many requests and report its latency keys (0: skip)")
    ap.add_argument("--high-contrast", type=int, default=1, choices=[0, 1],
                    help="cycles at viscosity ratio 1e3 on the 128x128x256 tube: rediscretised (gamma 1 and 0.7), "
                         "Galerkin, GCR(8) and both")
    ap.add_argument("--film", type=int, default=1, choices=[0, 1],
                    help="also step the 256x256x512 film once per solver and report its sweep fractions")
    ap.add_argument("--set", action="append", default=[], metavar="KEY=VALUE",
                    help="override a workload parameter (descriptor field), e.g. smoother_zblock=1")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("CSV", "OUT_MD"),
                    help="write the per-kernel summary of a rocprofv3 kernel-trace CSV and exit")
    ap.add_argument("--trace-command", default="", help="with --summarize-trace: the command that took the trace")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("PMC_DIR", "SITE", "LEVEL", "OUT_MD"),
                    help="write the traffic summary of a launch site from four rocprofv3 --pmc runs and exit")
    ap.add_argument("--counter-commands", action="append", default=[],
                    help="with --summarize-counters: the commands that took the counters (repeat)")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace[0], args.summarize_trace[1], args.workload, args.trace_command)
        return
    if args.summarize_counters:
        d, site, level, out = args.summarize_counters
        summarize_counters(d, args.workload, int(site), int(level), args.calibrate_copy or 256, args.counter_commands,
                           out)
        return
    if args.inner is None:
        args.inner = 2 if args.workload == "serving" else 4
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
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
    for kv in args.set:
        k, v = kv.split("=", 1)
        case["params"][k] = type(case["params"].get(k, 0))(float(v)) if k in case["params"] else int(v)
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
    serving = None
    if args.serving_requests > 0:
        sargs = argparse.Namespace(**vars(args))
        sargs.requests, sargs.inner, sargs.warmup = args.serving_requests, 2, 4
        sv = run_serving(sargs, log)
        serving = {k: sv[k] for k in ("value", "p50_step_ms", "p99_step_ms", "p50_request_s", "p99_request_s",
                                      "wall_s", "ticks", "peak_resident", "peak_bytes", "busy_dof_per_s",
                                      "failed_steps")}
        serving["unit"] = "DOF/s"
        serving["requests"] = args.serving_requests
        serving["rate_per_s"] = args.rate
        for k in ("steps", "ms_per_step", "group_build_s", "wall_outside_ticks_s", "slots", "group_builds",
                  "slots_given_back", "mean_resident", "p50_wait_s", "p99_wait_s"):
            if k in sv:
                serving[k] = sv[k]
    film = None
    if args.film:
        log("film3d_256x256x512: generating inputs")
        fcase = synth.WORKLOADS["film3d_256x256x512"]()
        film = {"grid": fcase["params"]["n"], "nodes": int(fcase["X"].shape[1])}
        fres = {}
        for m in ("fp64", "refined"):
            log(f"film, mode {m}: 1 warmup + 1 timed step + 1 kernel-timed step")
            fres[m] = run_mode(fcase, pkg.IBB_FP32_REFINED if m == "refined" else pkg.IBB_FP64, args.inner, 1, 1,
                               log, prof_steps=1)
            rows, _ = site_table(fres[m]["prof"], 3, 1)
            sites = {}
            for r in rows:
                if r["level"] == 0 and r["site"] in (0, 2, 4, 23, 24, 25, 26):
                    sites[r["kernel"]] = dict(avg_launch_us=round(r["avg_us"], 2), achieved=round(r["gbs"], 1),
                                              frac=round(r["gbs"] / HBM_PEAK_GBS, 4),
                                              algorithmic_bytes_per_launch=int(r["bytes_per_launch"]),
                                              share_of_step_kernels=round(r["share"], 4))
            film[m] = dict(dof_per_s=round(fres[m]["dof_per_s"], 1), ms_per_step=round(fres[m]["ms_per_step"], 3),
                           cycles_u=fres[m]["cycles_u"][0], cycles_p=fres[m]["cycles_p"][0],
                           largest_site=rows[0]["kernel"], level0=sites)
        film["refined_over_fp64"] = round(fres["refined"]["dof_per_s"] / fres["fp64"]["dof_per_s"], 3)
        del fcase
    high = None
    if args.high_contrast:
        # cycles to the tolerance at viscosity ratio 1e3 (FP64 V-cycles): the
        # coarse-operator remedies of Sec. "Numerical Concerns" side by side
        log("tube3d_128x128x256 (viscosity ratio 1e3): generating inputs")
        hcase = synth.WORKLOADS["tube3d_128x128x256"]()
        hp = hcase["params"]
        high = {"workload": "tube3d_128x128x256", "viscosity_ratio": hp["mu_max"] / hp["mu_out"],
                "precision": "fp64", "rtol": hp["rtol"], "steps": 2, "warmup": 1}
        variants = [("rediscretised_gamma_1", dict(gamma=[1.0] * 16), 0),
                    ("rediscretised_gamma_0.7", {}, 0),
                    ("galerkin", dict(galerkin=1), 0),
                    ("gcr8_gamma_0.7", {}, 8),
                    ("galerkin_gcr8", dict(galerkin=1), 8)]
        for name, over, kr in variants:
            log(f"high contrast, {name}: 1 warmup + 2 timed steps")
            r = run_mode(dict(hcase, params=dict(hp, **over)), pkg.IBB_FP64, 1, 2, 1, log, krylov=kr, prof_steps=1)
            build = r["prof"].get(27, None)
            build_ms = 0.0
            for cls, pr in r["prof"].items():
                if cls % 32 == 27:
                    build_ms += pr["total_ms"]
            high[name] = dict(mean_cycles_u=float(np.mean(r["cycles_u"])), mean_cycles_p=float(np.mean(r["cycles_p"])),
                              solve_ms_per_step=round(r["solve_ms"] / 2, 3), ms_per_step=round(r["ms_per_step"], 3),
                              dof_per_s=round(r["dof_per_s"], 1), max_relres=r["max_relres"])
            if build is not None or build_ms > 0:
                high[name]["galerkin_build_ms_per_step"] = round(build_ms, 3)
            high[name]["sites"] = [dict(kernel=t["kernel"], launches=t["launches"], avg_us=round(t["avg_us"], 2),
                                        ms_per_step=round(t["ms_per_step"], 3), share=round(t["share"], 4),
                                        frac=round(t["gbs"] / HBM_PEAK_GBS, 4))
                                   for t in site_table(r["prof"], 3, 1)[0][:8]]
        del hcase
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
    # roofline of the launch site with the largest device time per step in
    # the headline mode (kernel-by-kernel steps after the timed ones)
    D = p["dim"]
    rows, _ = site_table(head["prof"], D, args.steps)
    dom = rows[0]
    roof = dict(bound="hbm", achieved=round(dom["gbs"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(dom["gbs"] / HBM_PEAK_GBS, 4),
                traffic=committed_traffic(dom["site"], dom["level"], args.workload),
                kernel=dom["kernel"], avg_launch_us=round(dom["avg_us"], 2), launches=dom["launches"],
                algorithmic_bytes_per_launch=int(dom["bytes_per_launch"]),
                bytes_per_unit=words_per_unit(dom["site"], D) * SITES[dom["site"]][1],
                device_ms_per_step=round(dom["ms_per_step"], 3), share_of_step_kernels=round(dom["share"], 4))
    if dom["site"] in (12, 13, 14, 15, 16):
        roof["limited_by"] = "latency (one workgroup, barriers between passes)"
    rp = rocprof_average(p, dom["site"], dom["level"], args.workload)
    if rp:
        roof["rocprof_avg_launch_us"] = rp
        roof["rocprof_frac"] = round(dom["bytes_per_launch"] / (rp * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    # the finest-level viscous sweep of the headline mode (the pass the
    # bandwidth target is about), whether or not it dominates
    sw = next((r for r in rows if r["site"] == (2 if head_mode == "refined" else 0) and r["level"] == 0), None)
    sweep = None
    if sw:
        sweep = dict(kernel=sw["kernel"], achieved=round(sw["gbs"], 1), frac=round(sw["gbs"] / HBM_PEAK_GBS, 4),
                     avg_launch_us=round(sw["avg_us"], 2), algorithmic_bytes_per_launch=int(sw["bytes_per_launch"]),
                     device_ms_per_step=round(sw["ms_per_step"], 3), share_of_step_kernels=round(sw["share"], 4))
        rs = rocprof_average(p, sw["site"], sw["level"], args.workload)
        if rs:
            sweep["rocprof_avg_launch_us"] = rs
            sweep["rocprof_frac"] = round(sw["bytes_per_launch"] / (rs * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
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
                   "overrides": args.set or None,
                   "springs": int(case["ij"].shape[1]), "viscosity_ratio": p["mu_max"] / p["mu_out"],
                   "density_ratio": (p["rho0"] + p["rho_b"]) / p["rho0"], "rtol": p["rtol"],
                   "nu": [p["nu1"], p["nu2"]], "gamma_2h": p["gamma"][1], "precision": head_mode,
                   "inner_cycles": args.inner if head_mode == "refined" else None},
        "p50_step_ms": round(percentile(all_steps, 50), 3),
        "p99_step_ms": round(percentile(all_steps, 99), 3),
        "roofline": roof,
        "sweep": sweep,
        "cpu_baseline": cpu,
        "serving": serving,
        "film3d_256x256x512": film,
        "high_contrast": high,
    }
    for m in res:
        r = res[m]
        out[m] = dict(dof_per_s=round(r["dof_per_s"], 1), ms_per_step=round(r["ms_per_step"], 3),
                      solve_ms_per_step=round(r["solve_ms"] / args.steps, 3),
                      mean_cycles_u=float(np.mean(r["cycles_u"])), mean_cycles_p=float(np.mean(r["cycles_p"])),
                      mean_vcycles=float(np.mean(r["vcycles"])), max_relres=r["max_relres"],
                      p50_step_ms=round(percentile(r["step_ms"], 50), 3),
                      p99_step_ms=round(percentile(r["step_ms"], 99), 3),
                      sites=[dict(kernel=t["kernel"], launches=t["launches"], avg_us=round(t["avg_us"], 2),
                                  ms_per_step=round(t["ms_per_step"], 3), share=round(t["share"], 4),
                                  frac=round(t["gbs"] / HBM_PEAK_GBS, 4))
                             for t in site_table(r["prof"], D, args.steps)[0][:10]])
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
        refined_cv = "refined" in modes
        cv = {"viscosity_ratio": 1.0, "precision": head_mode}
        for dec, key in ((0, "coupled"), (1, "decoupled")):
            r = const[dec]
            sm = (20 if refined_cv else 19) if dec else (2 if refined_cv else 0)
            pr = r["prof"].get(sm, dict(launches=0, total_ms=0.0, units=0))
            avg_ms = pr["total_ms"] / max(pr["launches"], 1)
            bpl = words_per_unit(sm, D, bool(dec)) * SITES[sm][1] * pr["units"] / max(pr["launches"], 1)
            gbs = bpl / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
            cv[key] = dict(dof_per_s=round(r["dof_per_s"], 1), ms_per_step=round(r["ms_per_step"], 3),
                           solve_ms_per_step=round(r["solve_ms"] / args.steps, 3),
                           mean_cycles_u=float(np.mean(r["cycles_u"])), mean_cycles_p=float(np.mean(r["cycles_p"])),
                           max_relres=r["max_relres"],
                           smoother=dict(kernel=SITES[sm][0], launches=pr["launches"],
                                         avg_launch_us=round(avg_ms * 1e3, 2),
                                         algorithmic_bytes_per_launch=int(bpl), achieved_gbs=round(gbs, 1),
                                         frac=round(gbs / HBM_PEAK_GBS, 4)))
        cv["decoupled_over_coupled"] = round(const[1]["dof_per_s"] / const[0]["dof_per_s"], 3)
        out["constant_viscosity"] = cv
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
