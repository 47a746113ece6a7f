"""Groups (serving): contexts of different grids, dimensions, boundary kinds
and coefficients stepped together must give each member exactly the result
it gets when stepped alone, including members that join and leave between
steps (continuous batching), and a member that fails must not disturb the
others."""
import numpy as np
import pytest

from paper_1302_3663_amd import _lib as L
from paper_1302_3663_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def cases():
    return {
        "2d_periodic_walls": synth.tiny_2d(),
        "2d_inout_walls": synth.tiny_2d(inout=True),
        "3d_tube": synth.tiny_3d(),
        "3d_periodic_z": synth.tiny_3d(periodic_z=True),
        "channel2d_64x32": synth.channel_2d(seed=1),
        # a member whose V-cycle runs with launched passes down to its coarsest level
        "3d_tube_launched": dict(synth.tiny_3d(seed=5), params=dict(synth.tiny_3d(seed=5)["params"], wg_coarse_max=-1)),
        # a high-contrast member solved by GCR (its solves run on their own)
        "3d_tube_gcr": dict(synth.tiny_3d(seed=6), params=dict(synth.tiny_3d(seed=6)["params"], mu_max=1e3,
                                                                 krylov_restart=6)),
        # constant viscosity (eq:NSdis1): alone, one launch per colour covers
        # every component; in the group each component has its own pass
        "3d_tube_dec": dict(synth.tiny_3d(seed=7), params=dict(synth.tiny_3d(seed=7)["params"], mu_max=1.0,
                                                                 decoupled=1)),
        "2d_inout_dec": dict(synth.tiny_2d(inout=True, seed=8),
                             params=dict(synth.tiny_2d(inout=True, seed=8)["params"], mu_max=1.0, decoupled=1)),
    }


def make(case, precision):
    from paper_1302_3663_amd import ibmg
    return ibmg.from_case(case, precision=precision, inner_cycles=2)


def snapshot(ctx):
    u, p = ctx.get_state()
    X, F, alive = ctx.get_nodes()
    return [host(u), host(p), host(X), host(F), host(alive)]


def solo(case, precision, steps):
    ctx = make(case, precision)
    stats = []
    for _ in range(steps):
        s = ctx.projection_step()
        lag = ctx.lagrangian_update()
        stats.append((s["cycles_u"], s["cycles_p"], s["vcycles_u"], s["vcycles_p"], lag["n_broken"], lag["n_alive"]))
    out = snapshot(ctx)
    ctx.close()
    return out, stats


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("precision", [L.IBB_FP64, L.IBB_FP32_REFINED])
def test_group_equals_solo(precision):
    from paper_1302_3663_amd import ibmg
    cs = cases()
    names = sorted(cs)
    steps = 3
    ref = {n: solo(cs[n], precision, steps) for n in names}
    ctxs = [make(cs[n], precision) for n in names]
    g = ibmg.Group(ctxs)
    got = {n: [] for n in names}
    for _ in range(steps):
        ss = g.projection_step()
        ls = g.lagrangian_update()
        for n, s, lag in zip(names, ss, ls):
            assert s["relres_u"] <= 1e-10 and s["relres_p"] <= 1e-10
            got[n].append((s["cycles_u"], s["cycles_p"], s["vcycles_u"], s["vcycles_p"], lag["n_broken"],
                           lag["n_alive"]))
    for n, ctx in zip(names, ctxs):
        print("member", n, flush=True)
        assert got[n] == ref[n][1]
        assert same(snapshot(ctx), ref[n][0])
    g.close()
    for c in ctxs:
        c.close()


def test_members_join_and_leave():
    """Requests admitted at different ticks, in changing groups, each run
    their own number of steps; every result equals the request run alone."""
    from paper_1302_3663_amd import ibmg
    cs = cases()
    plan = {  # name: (tick of admission, steps)
        "3d_tube": (0, 3),
        "2d_inout_walls": (1, 2),
        "channel2d_64x32": (1, 3),
        "3d_periodic_z": (3, 1),
    }
    prec = L.IBB_FP32_REFINED
    ref = {n: solo(cs[n], prec, k)[0] for n, (_, k) in plan.items()}
    live, done, left = {}, {}, {}
    tick = 0
    while len(done) < len(plan):
        for n, (t0, k) in plan.items():
            if t0 == tick:
                live[n] = make(cs[n], prec)
                left[n] = k
        if live:
            names = sorted(live)
            print("tick", tick, "members", names, flush=True)
            g = ibmg.Group([live[n] for n in names])
            g.projection_step()
            g.lagrangian_update()
            g.close()
            for n in names:
                left[n] -= 1
                if left[n] == 0:
                    done[n] = snapshot(live[n])
                    live.pop(n).close()
        tick += 1
    for n in plan:
        assert same(done[n], ref[n]), n


def test_failing_member_is_isolated():
    from paper_1302_3663_amd import ibmg
    cs = cases()
    good = cs["3d_tube"]
    bad = dict(cs["2d_periodic_walls"])
    bad["params"] = dict(bad["params"], max_cycles=1)
    ref, _ = solo(good, L.IBB_FP64, 1)
    cg, cb = make(good, L.IBB_FP64), make(bad, L.IBB_FP64)
    g = ibmg.Group([cb, cg])
    with pytest.raises(L.IbbError) as e:
        g.projection_step()
    assert e.value.status == L.IBB_ENOCONV
    g.lagrangian_update()
    assert same(snapshot(cg), ref)
    g.close()
    cg.close()
    cb.close()


def test_group_rejects_mismatched_members():
    from paper_1302_3663_amd import ibmg
    cs = cases()
    a = make(cs["3d_tube"], L.IBB_FP64)
    b = make(cs["2d_periodic_walls"], L.IBB_FP32_REFINED)
    with pytest.raises(L.IbbError) as e:
        ibmg.Group([a, b])
    assert e.value.status == L.IBB_EINVAL
    with pytest.raises(L.IbbError) as e:
        ibmg.Group([a, a])
    assert e.value.status == L.IBB_EINVAL
    a.close()
    b.close()
