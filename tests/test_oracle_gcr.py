"""Pins of the oracle's V-cycle-preconditioned GCR against facts that do not
depend on its own code:
- GCR's k-th iterate minimises ||b - A x|| over x0 + span(z_1..z_k), where
  z_i = M r_{i-1} is one V-cycle on the previous residual: the first two
  iterates are recomputed here by least squares from the oracle's V-cycle and
  assembled matrix;
- the converged solution agrees with a sparse direct solve within cond * rtol;
- the residual does not increase from one iteration to the next within a
  restart window;
- at high viscosity contrast it needs fewer iterations than plain V-cycles."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from oracle import step as S
from paper_1302_3663_amd import synth


def state(case):
    st = S.State(case["params"], case["u0"], case["p0"], case["X"], case["ij"], case["rest"], case["K"])
    S.setup(st)
    return st


def to_vec(H, p, vel, compact):
    comp, pos = H.unknowns(vel)
    if vel:
        faces = O.split_faces(p, compact)
        return np.array([faces[a][k, j, i] for a, (i, j, k) in zip(comp, pos)])
    n = p["n"]
    arr = compact.reshape((n[2], n[1], n[0]) if p["dim"] == 3 else (1, n[1], n[0]))
    return np.array([arr[k, j, i] for (i, j, k) in pos])


def to_compact(H, p, vel, vec, template):
    out = np.array(template, dtype=np.float64, copy=True)
    comp, pos = H.unknowns(vel)
    if vel:
        faces = O.split_faces(p, out)
        for v, a, (i, j, k) in zip(vec, comp, pos):
            faces[a][k, j, i] = v
        return np.concatenate([f.ravel() for f in faces])
    n = p["n"]
    arr = out.reshape((n[2], n[1], n[0]) if p["dim"] == 3 else (1, n[1], n[0]))
    for v, (i, j, k) in zip(vec, pos):
        arr[k, j, i] = v
    return arr.ravel()


CASES = {
    "2d_periodic_walls": lambda: synth.tiny_2d(),
    "2d_inout_walls": lambda: synth.tiny_2d(inout=True),
    "3d_tube": lambda: synth.tiny_3d(),
}


def system(st, vel):
    p = st.p
    if vel:
        return O.momentum_rhs(p, st.u, st.rho, st.mu_c, st.mu_e, st.f), st.u
    b = O.pressure_rhs(p, st.u + 0.01 * np.random.default_rng(4).standard_normal(st.u.size))
    return b, np.zeros(b.size)


@pytest.mark.parametrize("name", sorted(CASES))
def test_first_iterates_minimise_the_residual(name):
    case = CASES[name]()
    p = case["params"]
    st = state(case)
    H = st.hier
    b, x0 = system(st, True)
    A = H.csr(True)
    bu, x0u = to_vec(H, p, True, b), to_vec(H, p, True, x0)
    r0 = bu - A @ x0u
    zero = np.zeros_like(x0)
    z1 = to_vec(H, p, True, H.vcycles(True, to_compact(H, p, True, r0, zero), zero, 1))
    q1 = A @ z1
    x1 = x0u + (r0 @ q1) / (q1 @ q1) * z1
    g1, _ = H.solve_gcr(True, b, x0, m=8, kmax=1)
    assert np.linalg.norm(to_vec(H, p, True, g1) - x1) <= 1e-12 * np.linalg.norm(x1)
    r1 = bu - A @ x1
    z2 = to_vec(H, p, True, H.vcycles(True, to_compact(H, p, True, r1, zero), zero, 1))
    Zm = np.stack([z1, z2], axis=1)
    c, *_ = np.linalg.lstsq(A @ Zm, r0, rcond=None)
    x2 = x0u + Zm @ c
    g2, _ = H.solve_gcr(True, b, x0, m=8, kmax=2)
    assert np.linalg.norm(to_vec(H, p, True, g2) - x2) <= 1e-10 * np.linalg.norm(x2)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("vel", [0, 1])
def test_converged_solution_matches_direct_solve(name, vel):
    case = CASES[name]()
    p = case["params"]
    st = state(case)
    H = st.hier
    b, x0 = system(st, bool(vel))
    x, info = H.solve_gcr(bool(vel), b, x0, m=8)
    assert info["status"] == 0 and info["relres"] <= p["rtol"]
    assert H.relres(bool(vel), b, x) <= p["rtol"] * (1 + 1e-6)
    A = H.csr(bool(vel))
    bu = to_vec(H, p, bool(vel), b)
    xu = to_vec(H, p, bool(vel), x)
    singular = (not vel) and not any(p["axis_bc"][a] == O.AX_INOUT for a in range(p["dim"]))
    if singular:
        Ad = A.toarray() + np.trace(A.toarray()) / A.shape[0] ** 2
        xs = np.linalg.solve(Ad, bu)
        xs, xu = xs - xs.mean(), xu - xu.mean()
    else:
        xs = spla.spsolve(A.tocsc(), bu)
    assert np.linalg.norm(xu - xs) <= 1e-8 * np.linalg.norm(xs)


def test_residual_does_not_increase():
    case = synth.tiny_3d()
    st = state(case)
    b, x0 = system(st, True)
    r0 = st.hier.relres(True, b, x0)
    rels = [r0] + [st.hier.solve_gcr(True, b, x0, m=8, kmax=k)[1]["relres"] for k in range(1, 8)]
    assert all(b_ <= a_ * (1 + 1e-12) for a_, b_ in zip(rels, rels[1:]))


def test_fewer_iterations_than_vcycles_at_high_contrast():
    case = synth.tiny_3d()
    case["params"] = dict(case["params"], mu_max=1e3)
    st = state(case)
    b, x0 = system(st, True)
    _, plain = st.hier.solve(True, b, x0)
    _, gcr = st.hier.solve_gcr(True, b, x0, m=8)
    assert gcr["status"] == 0 and plain["status"] == 0
    assert gcr["cycles"] < plain["cycles"]
