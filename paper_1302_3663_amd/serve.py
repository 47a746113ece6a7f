"""Continuous-batching request loop for independent biofilm solves.

Requests arrive over time and are served from a pool of slots: a slot is a
context of one problem shape (grid, boundary conditions, solver settings;
ibb_set_params lists what may differ between the problems of one shape),
with room for a given number of nodes and springs.  Every slot belongs to
one group, whose solve ticks are HIP graphs captured when the group is
built.  At every tick the loop
  1. admits, in arrival order, the requests that have arrived: a request
     goes into a free slot of its shape (reloaded in place, nothing is
     allocated or captured) and the slot is switched on in the group; when
     no such slot is free, the pool grows by one slot if the device-memory
     budget holds the new slot's workspace plus the workspace of the grown
     group (ibb_footprint_bytes, ibb_group_footprint_bytes) and the slot cap
     allows, after giving back free slots (least recently used first) as
     far as needed, and the group is built again; otherwise the request
     waits, and so do the ones behind it;
  2. steps every active slot once, together: one group projection step and
     one group Lagrangian update, whose multigrid passes share launches
     across the slots;
  3. retires the requests that have done their steps: their slots are
     switched off and free for the next admissions.
So the group is built again only when the pool changes; admissions and
retirements into slots of the right shape only switch slots.  Requests that
arrive while others are on the GPU join at the next tick.  Every request
computes exactly what it computes when run alone in a context of its own.
"""
import time

import numpy as np
import torch

from . import _lib as L
from . import ibmg

# descriptor fields that may differ between the problems of one slot
RELOADABLE = {"rho_b", "d0_pow_d", "mu_max", "break_ratio", "track_fragments", "attach_axis", "attach_dist",
              "rtol", "max_cycles"}


class Request:
    def __init__(self, rid, arrival, case, steps):
        self.rid = rid
        self.arrival = float(arrival)   # seconds after the start of the stream
        self.case = case
        self.steps = int(steps)
        self.footprint = 0
        self.slot = None
        self.admitted = None
        self.finished = None
        self.done = 0
        self.step_ms = []
        self.dof = 0
        self.solve_dof = 0                # DOF of every solve taken, summed
        self.status = []
        self.cycles = []
        self.final = None


class Slot:
    """A context of one problem shape with room for `capacity` nodes and
    springs; `req` is the request it holds (None: free)."""

    def __init__(self, key, ctx, capacity, footprint):
        self.key = key
        self.ctx = ctx
        self.capacity = capacity
        self.footprint = footprint
        self.req = None
        self.last_used = 0              # tick of the slot's last admission


def poisson_arrivals(n, rate, seed=0):
    """Arrival times of n requests with exponential gaps of mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def _frozen(v):
    if isinstance(v, (list, tuple, np.ndarray)):
        return tuple(_frozen(x) for x in v)
    return v


class Server:
    """krylov > 0: requests whose viscosity ratio is at least krylov_ratio are
    solved by V-cycle-preconditioned GCR(krylov); the rest by plain V-cycles,
    which share launches across the resident requests.  node_capacity and
    spring_capacity: the least room a new slot gets (a request that needs
    more gets a slot of its own size).  max_slots caps the pool (None: only
    the budget does); max_active caps the requests stepped together (None:
    no cap), a scheduling choice: larger ticks share more launches but every
    request in them waits for the slowest.  The pool outlives run(), so a
    warm-up stream leaves its slots to the next one; close() frees it."""

    def __init__(self, budget_bytes=32 << 30, max_slots=None, precision=L.IBB_FP32_REFINED, inner_cycles=2,
                 device="cuda:0", krylov=0, krylov_ratio=100.0, node_capacity=10000, spring_capacity=None,
                 max_active=None):
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.max_active = max_active
        self.slots = []
        self.group = None
        self.group_bytes = 0
        self.precision = precision
        self.inner = inner_cycles
        self.device = device
        self.krylov = int(krylov)
        self.krylov_ratio = float(krylov_ratio)
        self.node_capacity = int(node_capacity)
        self.spring_capacity = spring_capacity

    def request_case(self, case):
        p = case["params"]
        m = self.krylov if self.krylov > 0 and p["mu_max"] / p["mu_out"] >= self.krylov_ratio else 0
        return dict(case, params=dict(p, krylov_restart=m))

    def shape_key(self, case):
        p = self.request_case(case)["params"]
        return tuple(sorted((k, _frozen(v)) for k, v in p.items() if k not in RELOADABLE))

    def needs(self, case):
        return max(case["X"].shape[1], 1), max(case["ij"].shape[1], 1)

    def capacity_for(self, case):
        eta, m = self.needs(case)
        nodes = max(eta, self.node_capacity)
        springs = max(m, self.spring_capacity if self.spring_capacity is not None else 16 * nodes)
        return nodes, springs

    def footprint(self, case):
        """Workspace of a slot made for this case."""
        c = self.request_case(case)
        nodes, springs = self.capacity_for(case)
        return ibmg.footprint_bytes(c["params"], nodes, springs, self.precision, self.inner)

    def close(self):
        """Free the pool (and its group)."""
        if self.group is not None:
            self.group.close()
            self.group, self.group_bytes = None, 0
        for s in self.slots:
            s.ctx.close()
        self.slots = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, requests, keep_state=False, log=None):
        """Serve the requests (sorted by arrival) with the pool as it stands;
        returns a summary dict."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            r.footprint = self.footprint(r.case)
            if r.footprint > self.budget:
                raise ValueError(f"request {r.rid} needs {r.footprint} bytes, above the budget {self.budget}")
        slots, finished = self.slots, []
        used = sum(s.footprint for s in slots)   # workspaces of the slots
        group, group_bytes = self.group, self.group_bytes
        peak_used, peak_live = 0, 0
        ticks, tick_sizes, busy, build_s, builds, evicted = 0, [], 0.0, 0.0, 0, 0
        t0 = time.perf_counter()
        while pending or any(s.req is not None for s in slots):
            now = time.perf_counter() - t0
            ts = time.perf_counter()       # a tick runs from its admissions to the end of its step
            grew = False                   # the pool changed: the group is built again
            while pending and pending[0].arrival <= now:
                if self.max_active is not None and sum(1 for s in slots if s.req is not None) >= self.max_active:
                    break
                r = pending[0]
                key, need = self.shape_key(r.case), self.needs(r.case)
                slot = next((s for s in slots if s.req is None and s.key == key and s.capacity[0] >= need[0]
                             and s.capacity[1] >= need[1]), None)
                if slot is None:
                    c = self.request_case(r.case)
                    cap = self.capacity_for(r.case)

                    def give_back():
                        # the free slot used longest ago goes (the group, whose
                        # graphs use its arrays, goes first)
                        nonlocal group, group_bytes, used, evicted, grew
                        if group is not None:
                            group.close()
                            group, group_bytes = None, 0
                        old = min((s for s in slots if s.req is None), key=lambda s: s.last_used)
                        slots.remove(old)
                        old.ctx.close()
                        used -= old.footprint
                        evicted += 1
                        grew = True

                    # room by the slot cap and the slots' budget first, so that a
                    # request that must wait creates nothing
                    while ((self.max_slots is not None and len(slots) >= self.max_slots)
                           or used + r.footprint > self.budget) and any(s.req is None for s in slots):
                        give_back()
                    if (self.max_slots is not None and len(slots) >= self.max_slots) or \
                            used + r.footprint > self.budget:
                        if not any(s.req is not None for s in slots):
                            raise ValueError(f"request {r.rid} needs {r.footprint} bytes, above the budget "
                                             f"{self.budget}")
                        break
                    ctx = ibmg.Context(c["params"], cap[0], cap[1], self.precision, self.inner, self.device)
                    # then the group's workspace, which needs the context
                    while True:
                        gb = ibmg.group_footprint_bytes([s.ctx for s in slots] + [ctx])
                        fits = used + r.footprint + gb <= self.budget
                        if fits or not any(s.req is None for s in slots):
                            break
                        give_back()
                    if not fits:
                        ctx.close()
                        if not any(s.req is not None for s in slots):
                            raise ValueError(f"request {r.rid} with its group workspace needs "
                                             f"{r.footprint + gb} bytes, above the budget {self.budget}")
                        break
                    slot = Slot(key, ctx, cap, r.footprint)
                    slots.append(slot)
                    used += r.footprint
                    grew = True
                pending.pop(0)
                slot.ctx.load(self.request_case(r.case))
                slot.req = r
                slot.last_used = ticks
                r.slot = slot
                r.admitted = time.perf_counter() - t0
                r.dof = slot.ctx.n_face + slot.ctx.n_cell
                if group is not None and not grew:
                    group.set_active(slots.index(slot), True)
            live = [s for s in slots if s.req is not None]
            if not live:
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                continue
            if grew or group is None:
                tb = time.perf_counter()
                if group is not None:
                    group.close()
                    group = None
                group = ibmg.Group([s.ctx for s in slots])
                group_bytes = group.nbytes
                for i, s in enumerate(slots):
                    if s.req is None:
                        group.set_active(i, False)
                build_s += time.perf_counter() - tb
                builds += 1
            peak_used = max(peak_used, used + group_bytes)
            peak_live = max(peak_live, len(live))
            ss = group.projection_step(check=False)
            group.lagrangian_update()
            torch.cuda.synchronize(self.device)
            te = time.perf_counter()
            ticks += 1
            busy += te - ts
            tick_sizes.append(len(live))
            for i, s in enumerate(slots):
                r = s.req
                if r is None:
                    continue
                st = ss[i]
                r.step_ms.append(1e3 * (te - ts))
                r.status.append((st["status_u"], st["status_p"]))
                r.cycles.append((st["cycles_u"], st["cycles_p"]))
                r.solve_dof += st["dof_u"] + st["dof_p"]
                r.done += 1
            if log:
                log(f"tick {ticks}: {len(live)} resident of {len(slots)} slots, {1e3 * (te - ts):.1f} ms, "
                    f"{len(pending)} waiting, {len(finished)} done")
            for i, s in enumerate(slots):
                r = s.req
                if r is None or r.done < r.steps:
                    continue
                r.finished = time.perf_counter() - t0
                if keep_state:
                    u, p = s.ctx.get_state()
                    X, F, alive = s.ctx.get_nodes()
                    torch.cuda.synchronize(self.device)
                    r.final = [t.cpu().numpy() for t in (u, p, X, F, alive)]
                finished.append(r)
                s.req = None
                r.slot = None
                group.set_active(i, False)
        self.group, self.group_bytes = group, group_bytes
        wall = time.perf_counter() - t0
        steps = np.array([ms for r in finished for ms in r.step_ms])
        lat = np.array([r.finished - r.arrival for r in finished])
        waits = np.array([r.admitted - r.arrival for r in finished])
        dof = float(sum(r.solve_dof for r in finished))
        failed = sum(1 for r in finished for su, sp in r.status if su or sp)
        return dict(
            requests=len(finished), wall_s=wall, ticks=ticks,
            mean_resident=float(np.mean(tick_sizes)) if tick_sizes else 0.0, peak_resident=peak_live,
            peak_bytes=peak_used, slots=len(slots), group_builds=builds, slots_given_back=evicted,
            p50_step_ms=float(np.percentile(steps, 50)), p99_step_ms=float(np.percentile(steps, 99)),
            p50_request_s=float(np.percentile(lat, 50)), p99_request_s=float(np.percentile(lat, 99)),
            p50_wait_s=float(np.percentile(waits, 50)), p99_wait_s=float(np.percentile(waits, 99)),
            solve_dof_per_s=dof / wall, busy_s=busy, busy_dof_per_s=dof / busy if busy > 0 else 0.0,
            failed_steps=failed, group_build_s=build_s, wall_outside_ticks_s=wall - busy,
        )
