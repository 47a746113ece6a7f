"""Galerkin coarse operators of the viscous system on the GPU against the
oracle's (R A P assembled from its own transfers, Sec. "Numerical
Concerns"), through the C interface: V-cycle iterates after 1 and 3 cycles,
solves to the tolerance with the oracle's cycle counts, full projection
steps, the refined solver, GCR on top, and a high-contrast tube where the
Galerkin levels must cut the cycle count.  FP64 results within 1e-12
relative (2-norm and max norm)."""
import numpy as np
import pytest

import oracle as O
from oracle import step as S
from paper_1302_3663_amd import _lib as L
from paper_1302_3663_amd import synth

from parity import rel  # larger of the relative 2-norm and max-norm differences

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


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


def galerkin_case(name, **over):
    case = CASES[name]()
    case["params"] = dict(case["params"], galerkin=1, **over)
    return case


def oracle_state(case):
    st = S.State(case["params"], case["u0"], case["p0"], case["X"], case["ij"], case["rest"], case["K"])
    S.setup(st)
    return st


@pytest.mark.parametrize("name", sorted(CASES))
def test_vcycle_iterates_and_solve(name):
    from paper_1302_3663_amd import ibmg
    print("case", name, flush=True)
    case = galerkin_case(name)
    ctx = ibmg.from_case(case)
    st = oracle_state(case)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(ctx.n_face)
    x0 = case["u0"] + 0.1 * rng.standard_normal(ctx.n_face)
    for k in (1, 3):
        xg, _ = ctx.mg_solve(1, dev(b), dev(x0), exact=k)
        xo = st.hier.vcycles(True, b, x0, k)
        assert rel(host(xg), xo) < TOL, (k, rel(host(xg), xo))
    bm = O.momentum_rhs(case["params"], st.u, st.rho, st.mu_c, st.mu_e, st.f)
    xg, ig = ctx.mg_solve(1, dev(bm), dev(st.u))
    xo, io = st.hier.solve(True, bm, st.u)
    assert ig["cycles"] == io["cycles"], (ig, io)
    assert rel(host(xg), xo) < TOL
    ctx.close()


@pytest.mark.parametrize("name,steps", [("2d_inout_walls", 4), ("3d_tube", 3), ("3d_periodic_z", 2),
                                        ("channel2d_64x32", 5)])
def test_full_steps(name, steps):
    from paper_1302_3663_amd import ibmg
    print("case", name, "steps", steps, flush=True)
    case = galerkin_case(name)
    ctx = ibmg.from_case(case)
    st = oracle_state(case)
    for n in range(steps):
        sg = ctx.projection_step()
        so = S.projection_step(st)
        assert sg["cycles_u"] == so["u"]["cycles"] and sg["cycles_p"] == so["p"]["cycles"], (n, sg, so["u"])
        ctx.lagrangian_update()
        S.lagrangian_update(st)
    u, pr = ctx.get_state()
    X, F, _ = ctx.get_nodes()
    assert rel(host(u), st.u) < TOL
    assert rel(host(pr), st.pres) < TOL
    assert rel(host(X), st.X) < TOL
    ctx.close()


@pytest.mark.parametrize("name", ["3d_tube", "channel2d_64x32"])
def test_refined_and_gcr(name):
    """FP32 V-cycles on the FP32 copies of the Galerkin operators inside the
    FP64 correction reach the tolerance under the oracle's operator; GCR
    preconditioned by the Galerkin V-cycle takes the oracle's iterations."""
    from paper_1302_3663_amd import ibmg
    print("case", name, flush=True)
    case = galerkin_case(name)
    st = oracle_state(case)
    p = case["params"]
    bm = O.momentum_rhs(p, st.u, st.rho, st.mu_c, st.mu_e, st.f)
    ctx = ibmg.from_case(case, precision=L.IBB_FP32_REFINED, inner_cycles=2)
    xg, ig = ctx.mg_solve(1, dev(bm), dev(st.u))
    assert ig["relres"] <= p["rtol"]
    assert st.hier.relres(True, bm, host(xg)) <= p["rtol"] * (1 + 1e-6)
    ctx.close()
    case_k = galerkin_case(name, krylov_restart=6)
    ctx = ibmg.from_case(case_k)
    stk = oracle_state(case_k)
    xg, ig = ctx.mg_solve(1, dev(bm), dev(st.u))
    xo, io = stk.hier.solve_gcr(True, bm, st.u, m=6)
    assert ig["cycles"] == io["cycles"], (ig, io)
    assert rel(host(xg), xo) < 1e-11
    ctx.close()


def test_high_contrast_tube_cycles():
    """32x32x64 tube at mu_max / mu_out = 1e3: the GPU takes the oracle's
    Galerkin cycle count, and fewer cycles than with rediscretised coarse
    operators (gamma = 1)."""
    from paper_1302_3663_amd import ibmg
    base = synth.tube_3d(seed=3, n=(32, 32, 64), eta=1500, spacing=0.04, cutoff=0.1, rho_b=0.2, mu_max=1e3,
                         omega=0.02)
    cycles = {}
    for gal in (0, 1):
        case = dict(base, params=dict(base["params"], galerkin=gal, gamma=[1.0] * 16))
        print("galerkin", gal, flush=True)
        ctx = ibmg.from_case(case)
        st = oracle_state(case)
        p = case["params"]
        bm = O.momentum_rhs(p, st.u, st.rho, st.mu_c, st.mu_e, st.f)
        xg, ig = ctx.mg_solve(1, dev(bm), dev(st.u))
        if gal:
            xo, io = st.hier.solve(True, bm, st.u)
            assert ig["cycles"] == io["cycles"], (ig, io)
            assert rel(host(xg), xo) < TOL
        assert ig["relres"] <= p["rtol"]
        cycles[gal] = ig["cycles"]
        ctx.close()
    print("cycles rediscretised / galerkin", cycles, flush=True)
    assert cycles[1] < cycles[0]


def test_refused_in_groups_and_with_constant_viscosity():
    from paper_1302_3663_amd import ibmg
    case = galerkin_case("2d_inout_walls")
    ctx = ibmg.from_case(case)
    other = ibmg.from_case(CASES["2d_inout_walls"]())
    with pytest.raises(L.IbbError) as e:
        ibmg.Group([other, ctx])
    assert e.value.status == L.IBB_EINVAL
    ctx.close()
    other.close()
    p = dict(case["params"], decoupled=1, mu_max=case["params"]["mu_out"])
    with pytest.raises(L.IbbError) as e:
        ibmg.Context(p, 4, 4)
    assert e.value.status == L.IBB_EINVAL
