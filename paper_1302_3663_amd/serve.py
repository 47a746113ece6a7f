"""Continuous-batching request loop for independent biofilm solves.

Requests arrive over time.  At every tick the loop
  1. admits, in arrival order, the requests that have arrived, while the slot
     cap and the device-memory budget allow: the budget covers every resident
     request's workspace (ibb_footprint_bytes) plus the workspace of the group
     that steps them together (ibb_group_footprint_bytes); a request that does
     not fit waits, and so do the ones behind it;
  2. steps every resident request once, together: one group projection step
     and one group Lagrangian update, whose multigrid passes share launches
     across the requests and whose solve ticks are replayed HIP graphs;
  3. retires the requests that have done their steps, which frees their slot
     and memory for the next admissions.
Requests that arrive while others are on the GPU therefore join at the next
tick, and their work overlaps on the device with the work already there.
Every request computes exactly what it computes when run alone.
"""
import time

import numpy as np
import torch

from . import _lib as L
from . import ibmg


class Request:
    def __init__(self, rid, arrival, case, steps):
        self.rid = rid
        self.arrival = float(arrival)   # seconds after the start of the stream
        self.case = case
        self.steps = int(steps)
        self.footprint = 0
        self.ctx = None
        self.admitted = None
        self.finished = None
        self.done = 0
        self.step_ms = []
        self.dof = 0
        self.solve_dof = 0                # DOF of every solve taken, summed
        self.status = []
        self.cycles = []
        self.final = None


def poisson_arrivals(n, rate, seed=0):
    """Arrival times of n requests with exponential gaps of mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


class Server:
    """krylov > 0: requests whose viscosity ratio is at least krylov_ratio are
    solved by V-cycle-preconditioned GCR(krylov); the rest by plain V-cycles,
    which share launches across the resident requests."""

    def __init__(self, budget_bytes=32 << 30, max_slots=32, precision=L.IBB_FP32_REFINED, inner_cycles=2,
                 device="cuda:0", krylov=0, krylov_ratio=100.0):
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.precision = precision
        self.inner = inner_cycles
        self.device = device
        self.krylov = int(krylov)
        self.krylov_ratio = float(krylov_ratio)

    def request_case(self, case):
        p = case["params"]
        m = self.krylov if self.krylov > 0 and p["mu_max"] / p["mu_out"] >= self.krylov_ratio else 0
        return dict(case, params=dict(p, krylov_restart=m))

    def footprint(self, case):
        c = self.request_case(case)
        return ibmg.footprint_bytes(c["params"], max(c["X"].shape[1], 1), max(c["ij"].shape[1], 1), self.precision,
                                    self.inner)

    def run(self, requests, keep_state=False, log=None):
        """Serve the requests (sorted by arrival); returns a summary dict."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            r.footprint = self.footprint(r.case)
            if r.footprint > self.budget:
                raise ValueError(f"request {r.rid} needs {r.footprint} bytes, above the budget {self.budget}")
        live, finished = [], []
        used = 0                        # workspaces of the resident requests
        group_bytes = 0                 # workspace of the current group
        peak_used, peak_live = 0, 0
        group, members = None, ()
        ticks, tick_sizes, busy, build_s = 0, [], 0.0, 0.0
        t0 = time.perf_counter()
        while pending or live:
            now = time.perf_counter() - t0
            ts = time.perf_counter()       # a tick runs from its admissions to the end of its step
            while (pending and pending[0].arrival <= now and len(live) < self.max_slots
                   and used + pending[0].footprint <= self.budget):
                r = pending[0]
                ctx = ibmg.from_case(self.request_case(r.case), precision=self.precision,
                                     inner_cycles=self.inner, device=self.device)
                gb = ibmg.group_footprint_bytes([q.ctx for q in live] + [ctx])
                if used + r.footprint + gb > self.budget:
                    ctx.close()
                    if not live:
                        raise ValueError(f"request {r.rid} with its group workspace needs {r.footprint + gb} "
                                         f"bytes, above the budget {self.budget}")
                    break
                pending.pop(0)
                r.ctx = ctx
                r.admitted = time.perf_counter() - t0
                r.dof = r.ctx.n_face + r.ctx.n_cell
                used += r.footprint
                live.append(r)
            if not live:
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                continue
            ids = tuple(r.rid for r in live)
            if ids != members:
                tb = time.perf_counter()
                if group is not None:
                    group.close()
                group = ibmg.Group([r.ctx for r in live])
                group_bytes = group.nbytes
                members = ids
                build_s += time.perf_counter() - tb
            peak_used = max(peak_used, used + group_bytes)
            peak_live = max(peak_live, len(live))
            ss = group.projection_step(check=False)
            group.lagrangian_update()
            torch.cuda.synchronize(self.device)
            te = time.perf_counter()
            ticks += 1
            busy += te - ts
            tick_sizes.append(len(live))
            for r, s in zip(live, ss):
                r.step_ms.append(1e3 * (te - ts))
                r.status.append((s["status_u"], s["status_p"]))
                r.cycles.append((s["cycles_u"], s["cycles_p"]))
                r.solve_dof += s["dof_u"] + s["dof_p"]
                r.done += 1
            if log:
                log(f"tick {ticks}: {len(live)} resident, {1e3 * (te - ts):.1f} ms, "
                    f"{len(pending)} waiting, {len(finished)} done")
            still = []
            for r in live:
                if r.done >= r.steps:
                    r.finished = time.perf_counter() - t0
                    if keep_state:
                        u, p = r.ctx.get_state()
                        X, F, alive = r.ctx.get_nodes()
                        torch.cuda.synchronize(self.device)
                        r.final = [t.cpu().numpy() for t in (u, p, X, F, alive)]
                    used -= r.footprint
                    finished.append(r)
                else:
                    still.append(r)
            if len(still) != len(live):
                if group is not None:
                    group.close()
                    group, members, group_bytes = None, (), 0
                for r in live:
                    if r.finished is not None:
                        r.ctx.close()
                        r.ctx = None
            live = still
        if group is not None:
            group.close()
        wall = time.perf_counter() - t0
        steps = np.array([ms for r in finished for ms in r.step_ms])
        lat = np.array([r.finished - r.arrival for r in finished])
        waits = np.array([r.admitted - r.arrival for r in finished])
        dof = float(sum(r.solve_dof for r in finished))
        failed = sum(1 for r in finished for su, sp in r.status if su or sp)
        return dict(
            requests=len(finished), wall_s=wall, ticks=ticks,
            mean_resident=float(np.mean(tick_sizes)) if tick_sizes else 0.0, peak_resident=peak_live,
            peak_bytes=peak_used,
            p50_step_ms=float(np.percentile(steps, 50)), p99_step_ms=float(np.percentile(steps, 99)),
            p50_request_s=float(np.percentile(lat, 50)), p99_request_s=float(np.percentile(lat, 99)),
            p50_wait_s=float(np.percentile(waits, 50)), p99_wait_s=float(np.percentile(waits, 99)),
            solve_dof_per_s=dof / wall, busy_s=busy, busy_dof_per_s=dof / busy if busy > 0 else 0.0,
            failed_steps=failed, group_build_s=build_s, wall_outside_ticks_s=wall - busy,
        )
