"""Host logic of the serving loop (paper_1302_3663_amd/serve.py) on the CPU,
with stand-in contexts and groups: every request is served, slots of a shape
are reused without building the group again, the concurrency and slot caps
and the budget hold, free slots of other shapes are given back when the pool
is full (so a stream always drains), and at every step exactly the slots
that hold a request are switched on in the group."""
import types

import numpy as np
import pytest

from paper_1302_3663_amd import serve, synth


class FakeCtx:
    instances = 0

    def __init__(self, params, nodes, springs, *args):
        FakeCtx.instances += 1
        self.params = params
        self.capacity = (nodes, springs)
        self.n_face, self.n_cell = 10, 5
        self.loaded = False
        self.closed = False

    def load(self, case):
        assert not self.closed
        assert case["X"].shape[1] <= self.capacity[0] and case["ij"].shape[1] <= self.capacity[1]
        self.loaded = True

    def close(self):
        self.closed = True


class FakeGroup:
    builds = 0

    def __init__(self, ctxs):
        FakeGroup.builds += 1
        assert all(not c.closed for c in ctxs)
        self.ctxs = ctxs
        self.active = [True] * len(ctxs)
        self.nbytes = 1000 * len(ctxs)
        self.closed = False

    def set_active(self, i, a):
        assert not self.closed
        self.active[i] = bool(a)
        if not a:
            self.ctxs[i].loaded = False

    def projection_step(self, check=False):
        assert not self.closed
        # exactly the slots holding a request take part
        assert self.active == [c.loaded for c in self.ctxs]
        return [dict(status_u=0, status_p=0, cycles_u=1 if a else 0, cycles_p=1 if a else 0,
                     dof_u=10 if a else 0, dof_p=5 if a else 0) for a in self.active]

    def lagrangian_update(self):
        pass

    def close(self):
        self.closed = True


@pytest.fixture
def fake(monkeypatch):
    FakeGroup.builds = 0
    FakeCtx.instances = 0
    fp = {"slot": 10 ** 6}
    monkeypatch.setattr(serve, "ibmg", types.SimpleNamespace(
        Context=FakeCtx, Group=FakeGroup, footprint_bytes=lambda *a, **k: fp["slot"],
        group_footprint_bytes=lambda ctxs: 1000 * len(ctxs)))
    monkeypatch.setattr(serve, "torch", types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda *a: None)))
    return fp


def mixed_cases():
    return [synth.tiny_2d(), synth.tiny_3d(), synth.tiny_2d(inout=True), synth.channel_2d(seed=1),
            synth.tiny_3d(periodic_z=True)]


def test_same_shape_reuses_slots(fake):
    cases = [synth.tiny_3d(seed=s) for s in range(6)]
    reqs = [serve.Request(i, 0.0, c, 2) for i, c in enumerate(cases)]
    srv = serve.Server(budget_bytes=1 << 30, max_slots=2)
    out = srv.run(reqs)
    assert out["requests"] == 6 and out["slots"] == 2 and out["group_builds"] == 1
    assert FakeCtx.instances == 2 and all(r.done == 2 for r in reqs)
    # the pool outlives the stream: a second one builds nothing
    more = [serve.Request(10 + i, 0.0, c, 1) for i, c in enumerate(cases[:3])]
    out2 = srv.run(more)
    assert out2["group_builds"] == 0 and FakeCtx.instances == 2
    srv.close()


@pytest.mark.parametrize("max_slots", [1, 2, 3])
def test_full_pool_gives_back_free_slots(fake, max_slots):
    """Shapes outnumber the slot cap: free slots of other shapes are given
    back (least recently used first), and the stream drains."""
    cases = mixed_cases() * 3
    reqs = [serve.Request(i, 0.0, c, 2) for i, c in enumerate(cases)]
    srv = serve.Server(budget_bytes=1 << 30, max_slots=max_slots)
    out = srv.run(reqs)
    srv.close()
    assert out["requests"] == len(reqs) and out["slots"] <= max_slots
    assert out["peak_resident"] <= max_slots and out["slots_given_back"] > 0


def test_concurrency_cap(fake):
    cases = mixed_cases() * 4
    reqs = [serve.Request(i, 0.0, c, 3) for i, c in enumerate(cases)]
    srv = serve.Server(budget_bytes=1 << 30, max_active=3)
    out = srv.run(reqs)
    srv.close()
    assert out["requests"] == len(reqs) and out["peak_resident"] <= 3


def test_budget_binds_pool(fake):
    """Budget for two slots plus the group's workspace: never more than two
    slots, and the peak accounting stays inside the budget."""
    fake["slot"] = 10 ** 6
    cases = [synth.tiny_3d(seed=s) for s in range(5)]
    reqs = [serve.Request(i, 0.0, c, 2) for i, c in enumerate(cases)]
    budget = 2 * 10 ** 6 + 2 * 1000 + 10
    srv = serve.Server(budget_bytes=budget)
    out = srv.run(reqs)
    srv.close()
    assert out["requests"] == 5 and out["slots"] == 2 and out["peak_bytes"] <= budget


def test_request_above_budget_is_refused(fake):
    fake["slot"] = 10 ** 9
    srv = serve.Server(budget_bytes=10 ** 6)
    with pytest.raises(ValueError):
        srv.run([serve.Request(0, 0.0, synth.tiny_2d(), 1)])


def test_larger_request_gets_its_own_slot(fake):
    small = synth.tiny_3d(seed=1)
    big = synth.tiny_3d(seed=2)
    big = dict(big, X=np.zeros((3, 20000)), ij=np.zeros((2, 10), np.int32))
    reqs = [serve.Request(0, 0.0, small, 1), serve.Request(1, 0.5, big, 1)]
    srv = serve.Server(budget_bytes=1 << 30, node_capacity=1000)
    out = srv.run(reqs)
    srv.close()
    assert out["requests"] == 2 and out["slots"] == 2
