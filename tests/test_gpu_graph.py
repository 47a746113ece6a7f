"""Solver iterations replayed as HIP graphs (the default) against the same
iterations launched one kernel at a time (the path taken while kernel timing
is on): identical bits and cycle counts over several steps, with the step's
own eager work and synchronisations between the replays.  Covers plain
V-cycles, refined outer iterations and GCR windows."""
import numpy as np
import pytest

from paper_1302_3663_amd import _lib as L
from paper_1302_3663_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


CASES = {
    "2d_inout_walls": lambda: synth.tiny_2d(inout=True),
    "3d_tube": lambda: synth.tiny_3d(),
    "3d_periodic_z": lambda: synth.tiny_3d(periodic_z=True),
    "channel2d_64x32": lambda: synth.channel_2d(seed=1),
    "3d_tube_launched": lambda: dict(synth.tiny_3d(seed=5),
                                     params=dict(synth.tiny_3d(seed=5)["params"], wg_coarse_max=-1)),
    "3d_tube_one_launch_sweep": lambda: dict(synth.tiny_3d(seed=6),
                                             params=dict(synth.tiny_3d(seed=6)["params"], smoother_passes=1,
                                                         wg_coarse_max=8)),
    # GCR with a short restart window: every window position has its own
    # graph, and each is replayed several times within a solve
    "3d_tube_gcr3": lambda: dict(synth.tiny_3d(seed=7),
                                 params=dict(synth.tiny_3d(seed=7)["params"], mu_max=1e3, krylov_restart=3)),
    "channel2d_gcr8": lambda: dict(synth.channel_2d(seed=1),
                                   params=dict(synth.channel_2d(seed=1)["params"], krylov_restart=8)),
}


def run(case, precision, timed):
    from paper_1302_3663_amd import ibmg
    ctx = ibmg.from_case(case, precision=precision, inner_cycles=2)
    ctx.profile_enable(timed)
    stats = []
    for _ in range(3):
        s = ctx.projection_step()
        ctx.lagrangian_update()
        stats.append((s["cycles_u"], s["cycles_p"], s["vcycles_u"], s["vcycles_p"], s["relres_u"], s["relres_p"]))
    u, p = ctx.get_state()
    X, F, _ = ctx.get_nodes()
    out = [host(u), host(p), host(X), host(F)]
    ctx.close()
    return out, stats


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", [L.IBB_FP64, L.IBB_FP32_REFINED])
def test_graph_equals_launches(name, precision):
    print("case", name, "precision", precision, flush=True)
    case = CASES[name]()
    ref, sref = run(case, precision, True)
    got, sgot = run(case, precision, False)
    assert sgot == sref
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_exact_cycles_through_graph():
    from paper_1302_3663_amd import ibmg
    case = synth.tiny_3d()
    outs = []
    for timed in (True, False):
        ctx = ibmg.from_case(case, precision=L.IBB_FP32_REFINED, inner_cycles=2)
        ctx.profile_enable(timed)
        rng = np.random.default_rng(1)
        b = torch.as_tensor(rng.standard_normal(ctx.n_face), device="cuda:0")
        x0 = torch.as_tensor(case["u0"], device="cuda:0")
        res = []
        for k in (1, 2, 5):
            x, info = ctx.mg_solve(1, b, x0, exact=k)
            res.append((host(x), info["cycles"], info["relres"]))
        outs.append(res)
        ctx.close()
    for (xa, ca, ra), (xb, cb, rb) in zip(*outs):
        assert ca == cb and ra == rb and np.array_equal(xa, xb)
