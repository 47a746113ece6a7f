"""Flow-level pins for the oracle's time step.

- 2D biofilm-free channel (periodic in x, walls in y, body force g): the
  steady state is the solution of the tridiagonal system
  -Re^-1 mu delta_yy u = g with zero velocity at the walls (odd ghosts),
  solved here by scipy.linalg.solve_banded, and the error of a run started
  at half the profile contracts per step by the factor
  1 / (1 + dt Re^-1 mu lambda_1 / sigma) of the slowest mode,
  lambda_1 = (4 / h^2) sin^2(pi h / (2 Ly)) (Sec. "Two-Dimensional
  Validation": convergence well within 300 steps at dt = 1e-4);
- 3D biofilm-free square duct (periodic along the axis, walls on the sides):
  the discrete steady state approaches the laminar series solution
  eq:3DlaminarFlow at O(h^2) (Sec. "Three-Dimensional Validation");
- projection identity: D u^{n+1} = -(eps dt / sigma) (b_p - A_p p), so the
  divergence after a step is the pressure residual (eq:NSdis2-eq:NSdis4).
"""
import math

import numpy as np
import scipy.linalg as sla

import oracle as O
from oracle import step as S
from paper_1302_3663_amd import synth


def no_biofilm_state(p, u0):
    X = np.zeros((p["dim"], 0))
    st = S.State(p, u0, np.zeros(O.cell_count(p)), X, np.zeros((2, 0), np.int32), np.zeros(0), np.zeros(0))
    S.setup(st)
    return st


def test_2d_laminar_steady_state_and_decay():
    ny, nx = 32, 8
    p = synth.base_params(2, [nx, ny], [O.AX_PERIODIC, O.AX_WALLS], 1.0 / ny)
    g = 8.0 * p["mu_out"] * p["inv_re"]
    p["body_force"] = [g, 0.0, 0.0]
    h = p["h"]
    # steady state: tridiagonal with odd ghosts at both walls
    c = p["inv_re"] * p["mu_out"] / h ** 2
    ab = np.zeros((3, ny))
    ab[0, 1:] = -c
    ab[1, :] = 2 * c
    ab[1, 0] += c
    ab[1, -1] += c
    ab[2, :-1] = -c
    us = sla.solve_banded((1, 1), ab, np.full(ny, g))
    u0 = 0.5 * synth.initial_velocity(p)
    st = no_biofilm_state(p, u0)
    errs = []
    for _ in range(60):
        S.projection_step(st)
        ux = O.split_faces(p, st.u)[0][0]
        errs.append(np.abs(ux - us[:, None]).max())
    lam1 = (4 / h ** 2) * math.sin(math.pi * h / 2) ** 2
    factor = 1.0 / (1.0 + p["dt"] * p["inv_re"] * p["mu_out"] * lam1 / p["sigma"])
    ratios = np.array(errs[10:40]) / np.array(errs[9:39])
    np.testing.assert_allclose(ratios, factor, rtol=1e-3)
    assert errs[-1] < 1e-8
    # the discrete steady state sits O(h^2) off the exact parabola, not on it
    y = (np.arange(ny) + 0.5) * h
    assert 1e-5 < np.abs(us - 4 * y * (1 - y)).max() < 10 * h * h


def duct_series(n, h, terms=301):
    """u(x, y) solving -Lap u = 1 in the unit square with u = 0 on the walls"""
    x = (np.arange(n) + 0.5) * h
    s = np.zeros((n, n))
    for a in range(1, terms + 1, 2):
        sx = np.sin(a * math.pi * x)
        for b in range(1, terms + 1, 2):
            s += np.outer(np.sin(b * math.pi * x), sx) / (a * b * (a * a + b * b))
    return 16.0 / math.pi ** 4 * s


def test_3d_duct_second_order():
    errs = []
    for n in (8, 16):
        h = 1.0 / n
        p = synth.base_params(3, [n, n, 4], [O.AX_WALLS, O.AX_WALLS, O.AX_PERIODIC], h)
        p["dt"] = 1e6            # the mass term vanishes: one step is the steady Stokes solve
        p["body_force"] = [0.0, 0.0, 1.0]
        st = no_biofilm_state(p, np.zeros(sum(O.face_counts(p))))
        S.projection_step(st)
        uz = O.split_faces(p, st.u)[2][0]
        want = duct_series(n, h) / (p["inv_re"] * p["mu_out"])
        errs.append(np.abs(uz - want).max() / want.max())
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


def test_projection_identity_and_divergence():
    for case in (synth.tiny_2d(), synth.tiny_2d(inout=True), synth.tiny_3d()):
        p = case["params"]
        st = S.State(p, case["u0"], case["p0"], case["X"], case["ij"], case["rest"], case["K"])
        S.setup(st)
        out = S.projection_step(st)
        div = O.divergence(p, st.u)
        Ap = st.hier.csr(False)
        r = out["b_p"] - Ap @ st.pres
        lhs = np.linalg.norm(div)
        rhs = p["eps"] * p["dt"] / p["sigma"] * np.linalg.norm(r)
        assert abs(lhs - rhs) <= 1e-6 * rhs + 1e-12
        assert np.linalg.norm(r) <= p["rtol"] * np.linalg.norm(out["b_p"]) * (1 + 1e-12)
