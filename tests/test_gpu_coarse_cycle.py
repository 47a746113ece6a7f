"""The coarse part of a V-cycle run inside one workgroup must take exactly the
passes of the launched kernels: iterates agree bit for bit with the launched
path (switch-over disabled), whatever level the switch happens at.  Applied as
its precomputed linear map (the tail below the workgroup's start level), the
same part agrees with the recursion up to rounding: 1e-13 relative in FP64,
1e-5 for the FP32 inner cycles of the refined solver."""
import numpy as np
import pytest

from paper_1302_3663_amd import _lib as L
from paper_1302_3663_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


CASES = {
    "2d_periodic_walls": lambda: synth.tiny_2d(),
    "2d_inout_walls": lambda: synth.tiny_2d(inout=True),
    "3d_tube": lambda: synth.tiny_3d(),
    "3d_periodic_z": lambda: synth.tiny_3d(periodic_z=True),
    "channel2d_64x32": lambda: synth.channel_2d(seed=1),
}


def run(case, wg, precision, tail=-1):
    from paper_1302_3663_amd import ibmg
    c = dict(case)
    c["params"] = dict(case["params"], wg_coarse_max=wg, coarse_tail=tail)
    ctx = ibmg.from_case(c, precision=precision, inner_cycles=2)
    rng = np.random.default_rng(7)
    out = []
    for vel, n in ((1, ctx.n_face), (0, ctx.n_cell)):
        b = rng.standard_normal(n)
        x0 = case["u0"] if vel else np.zeros(n)
        x, _ = ctx.mg_solve(vel, dev(b), dev(x0), exact=3)
        out.append(host(x))
    s = ctx.projection_step()
    u, p = ctx.get_state()
    out += [host(u), host(p)]
    ctx.close()
    return out, (s["cycles_u"], s["cycles_p"])


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", [L.IBB_FP64, L.IBB_FP32_REFINED])
@pytest.mark.parametrize("wg", [0, 64, 8])
def test_workgroup_cycle_matches_launched(name, precision, wg):
    print("case", name, "precision", precision, "wg", wg, flush=True)
    case = CASES[name]()
    ref, cyc_ref = run(case, -1, precision)
    got, cyc = run(case, wg, precision)
    assert cyc == cyc_ref
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", [L.IBB_FP64, L.IBB_FP32_REFINED])
@pytest.mark.parametrize("wg", [0, 64])
def test_tail_matches_recursion(name, precision, wg):
    from parity import rel
    print("case", name, "precision", precision, "wg", wg, flush=True)
    case = CASES[name]()
    ref, cyc_ref = run(case, wg, precision, tail=-1)
    got, cyc = run(case, wg, precision, tail=0)
    assert cyc == cyc_ref
    tol = 1e-13 if precision == L.IBB_FP64 else 1e-5
    errs = [rel(a, b) for a, b in zip(got, ref)]
    print("tail against recursion", errs, flush=True)
    assert max(errs) < tol


def run_passes(case, passes, precision, nu=(2, 2)):
    from paper_1302_3663_amd import ibmg
    c = dict(case)
    c["params"] = dict(case["params"], smoother_passes=passes, wg_coarse_max=8, nu1=nu[0], nu2=nu[1])
    ctx = ibmg.from_case(c, precision=precision, inner_cycles=2)
    rng = np.random.default_rng(9)
    out = []
    for vel, n in ((1, ctx.n_face), (0, ctx.n_cell)):
        b = rng.standard_normal(n)
        x0 = case["u0"] if vel else np.zeros(n)
        x, _ = ctx.mg_solve(vel, dev(b), dev(x0), exact=2)
        out.append(host(x))
    for _ in range(2):
        s = ctx.projection_step()
        ctx.lagrangian_update()
    u, p = ctx.get_state()
    out += [host(u), host(p)]
    ctx.close()
    return out, (s["cycles_u"], s["cycles_p"])


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", [L.IBB_FP64, L.IBB_FP32_REFINED])
@pytest.mark.parametrize("nu", [(2, 2), (3, 3), (1, 3)])
def test_one_launch_sweep_matches_two(name, precision, nu):
    """The one-launch red-black sweep (LDS tiles, second buffer) gives the
    bits of the two launches per sweep; a small workgroup budget keeps
    several levels on launched passes.  An odd number of pre-smoothing sweeps
    leaves the buffers exchanged during the coarse-grid correction."""
    print("case", name, "precision", precision, "nu", nu, flush=True)
    case = CASES[name]()
    ref, cyc_ref = run_passes(case, 2, precision, nu)
    got, cyc = run_passes(case, 1, precision, nu)
    assert cyc == cyc_ref
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_one_launch_sweep_full_size():
    from paper_1302_3663_amd import ibmg
    case = synth.WORKLOADS["tube3d_64x64x128"]()
    outs = []
    for passes in (2, 1):
        c = dict(case, params=dict(case["params"], smoother_passes=passes))
        ctx = ibmg.from_case(c, precision=L.IBB_FP32_REFINED, inner_cycles=2)
        s = ctx.projection_step()
        u, p = ctx.get_state()
        outs.append((host(u), host(p), s["cycles_u"], s["cycles_p"]))
        ctx.close()
    assert outs[0][2:] == outs[1][2:]
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def run_zblock(case, zb, precision, steps=2):
    from paper_1302_3663_amd import ibmg
    c = dict(case, params=dict(case["params"], smoother_zblock=zb))
    ctx = ibmg.from_case(c, precision=precision, inner_cycles=2)
    out, cyc = [], []
    for _ in range(steps):
        s = ctx.projection_step()
        ctx.lagrangian_update()
        cyc.append((s["cycles_u"], s["cycles_p"]))
    u, p = ctx.get_state()
    out += [host(u), host(p)]
    ctx.close()
    return out, cyc


@pytest.mark.parametrize("name", ["3d_tube", "3d_periodic_z", "tube3d_64x64x128"])
@pytest.mark.parametrize("precision", [L.IBB_FP64, L.IBB_FP32_REFINED])
def test_zblocked_passes_match_flat(name, precision):
    """Colour passes walked in z-blocks (a workgroup per band of rows and run
    of planes) give the bits of the flat passes (one point per thread)."""
    print("case", name, "precision", precision, flush=True)
    case = synth.WORKLOADS[name]() if name in synth.WORKLOADS else CASES[name]()
    ref, cyc_ref = run_zblock(case, -1, precision)
    got, cyc = run_zblock(case, 1, precision)
    assert cyc == cyc_ref
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
