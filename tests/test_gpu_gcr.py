"""GCR on the GPU (V-cycle-preconditioned, restarted after m directions)
against the oracle's GCR: iterates after exactly k iterations, converged
cycle counts and solutions, full steps; the refined variant (FP32 V-cycles as
the preconditioner) against the exact discrete solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from oracle import step as S
from paper_1302_3663_amd import _lib as L
from paper_1302_3663_amd import synth

from parity import rel  # larger of the relative 2-norm and max-norm differences

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M = 6


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


CASES = {
    "2d_periodic_walls": lambda: synth.tiny_2d(),
    "2d_inout_walls": lambda: synth.tiny_2d(inout=True),
    "3d_tube": lambda: synth.tiny_3d(),
    "3d_tube_mu1e3": lambda: dict(synth.tiny_3d(), params=dict(synth.tiny_3d()["params"], mu_max=1e3)),
    "channel2d_64x32": lambda: synth.channel_2d(seed=1),
}


def setup(name, precision=L.IBB_FP64):
    from paper_1302_3663_amd import ibmg
    case = CASES[name]()
    case["params"] = dict(case["params"], krylov_restart=M)
    ctx = ibmg.from_case(case, precision=precision, inner_cycles=2)
    st = S.State(case["params"], case["u0"], case["p0"], case["X"], case["ij"], case["rest"], case["K"])
    S.setup(st)
    return case, ctx, st


def unknown_vector(H, p, vel, compact):
    comp, pos = H.unknowns(vel)
    if vel:
        faces = O.split_faces(p, compact)
        return np.array([faces[a][k, j, i] for a, (i, j, k) in zip(comp, pos)])
    n = p["n"]
    arr = compact.reshape((n[2], n[1], n[0]) if p["dim"] == 3 else (1, n[1], n[0]))
    return np.array([arr[k, j, i] for (i, j, k) in pos])


def system(st, vel):
    p = st.p
    if vel:
        return O.momentum_rhs(p, st.u, st.rho, st.mu_c, st.mu_e, st.f), st.u
    b = O.pressure_rhs(p, st.u + 0.01 * np.random.default_rng(4).standard_normal(st.u.size))
    return b, np.zeros(b.size)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("vel", [0, 1])
@pytest.mark.parametrize("k", [1, 3, 8])
def test_iterates_match_oracle(name, vel, k):
    print("case", name, "velocity" if vel else "pressure", "iterations", k, flush=True)
    case, ctx, st = setup(name)
    b, x0 = system(st, bool(vel))
    xg, _ = ctx.mg_solve(vel, dev(b), dev(x0), exact=k)
    xo, _ = st.hier.solve_gcr(bool(vel), b, x0, m=M, kmax=k)
    assert rel(host(xg), xo) < 1e-11
    ctx.close()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("vel", [0, 1])
def test_converged_solve(name, vel):
    case, ctx, st = setup(name)
    p = case["params"]
    b, x0 = system(st, bool(vel))
    xg, ig = ctx.mg_solve(vel, dev(b), dev(x0))
    xo, io = st.hier.solve_gcr(bool(vel), b, x0, m=M)
    print("case", name, "velocity" if vel else "pressure", "gpu", ig, "oracle", io["cycles"], flush=True)
    assert ig["cycles"] == io["cycles"] and ig["relres"] <= p["rtol"]
    assert st.hier.relres(bool(vel), b, host(xg)) <= p["rtol"] * (1 + 1e-6)
    assert rel(host(xg), xo) < 1e-10
    ctx.close()


@pytest.mark.parametrize("name", ["3d_tube", "channel2d_64x32", "3d_tube_mu1e3"])
def test_full_steps(name):
    case, ctx, st = setup(name)
    for k in range(3):
        sg = ctx.projection_step()
        so = S.projection_step(st)
        assert sg["cycles_u"] == so["u"]["cycles"] and sg["cycles_p"] == so["p"]["cycles"]
        ctx.lagrangian_update()
        S.lagrangian_update(st)
    u, _ = ctx.get_state()
    assert rel(host(u), st.u) < 1e-10
    ctx.close()


@pytest.mark.parametrize("name", ["3d_tube", "2d_inout_walls", "3d_tube_mu1e3"])
@pytest.mark.parametrize("vel", [0, 1])
def test_refined_gcr_against_direct(name, vel):
    case, ctx, st = setup(name, precision=L.IBB_FP32_REFINED)
    p = case["params"]
    b, x0 = system(st, bool(vel))
    xg, ig = ctx.mg_solve(vel, dev(b), dev(x0))
    xg = host(xg)
    assert ig["relres"] <= p["rtol"]
    assert st.hier.relres(bool(vel), b, xg) <= p["rtol"] * (1 + 1e-6)
    A = st.hier.csr(bool(vel))
    bu = unknown_vector(st.hier, p, bool(vel), b)
    xu = unknown_vector(st.hier, p, bool(vel), xg)
    singular = (not vel) and not any(p["axis_bc"][a] == O.AX_INOUT for a in range(p["dim"]))
    if singular:
        Ad = A.toarray() + np.trace(A.toarray()) / A.shape[0] ** 2
        xs = np.linalg.solve(Ad, bu)
        xs, xu = xs - xs.mean(), xu - xu.mean()
    else:
        xs = spla.spsolve(A.tocsc(), bu)
    assert rel(xu, xs) < 1e-9
    ctx.close()


def test_fewer_iterations_than_vcycles():
    from paper_1302_3663_amd import ibmg
    case = CASES["3d_tube_mu1e3"]()
    plain = ibmg.from_case(case)
    case, gcr, st = setup("3d_tube_mu1e3")
    sp, sg = plain.projection_step(), gcr.projection_step()
    assert sg["cycles_u"] < sp["cycles_u"]
    plain.close()
    gcr.close()


def test_group_with_gcr_member_equals_solo():
    from paper_1302_3663_amd import ibmg
    _, solo_g, _ = setup("3d_tube_mu1e3")
    solo_p = ibmg.from_case(CASES["channel2d_64x32"]())
    s1, s2 = solo_g.projection_step(), solo_p.projection_step()
    _, gg, _ = setup("3d_tube_mu1e3")
    gp = ibmg.from_case(CASES["channel2d_64x32"]())
    grp = ibmg.Group([gg, gp])
    t1, t2 = grp.projection_step()
    assert (t1["cycles_u"], t1["cycles_p"], t2["cycles_u"], t2["cycles_p"]) == \
        (s1["cycles_u"], s1["cycles_p"], s2["cycles_u"], s2["cycles_p"])
    for a, b in ((solo_g, gg), (solo_p, gp)):
        ua, pa = a.get_state()
        ub, pb = b.get_state()
        assert np.array_equal(host(ua), host(ub)) and np.array_equal(host(pa), host(pb))
    grp.close()
    for c in (solo_g, solo_p, gg, gp):
        c.close()
