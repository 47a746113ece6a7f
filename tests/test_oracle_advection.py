"""Pins for the oracle's explicit advection term of eq:NSdis1-1, the
skew-symmetric form 1/2 (u . D0 u_a + D0 . (u u_a)) read on the MAC lattice
(each a-face uses the average of the four surrounding b-faces for u_b, b != a,
and central differences over 2h; one layer beyond a fixed face is the odd
reflection through the face value, beyond the outflow face the even mirror).

The term is read back from the momentum right-hand side with unit density,
no force, no body force and no boundary term:
b_a = sigma u_a / dt - N_a, so N_a = sigma u_a / dt - b_a.

- Polynomial exactness.  For a linear velocity the four-point average is
  exact, central differences are exact on the quadratic products, so at
  every face whose stencil stays inside the stored domain N_a equals the
  continuum value u . grad u_a + 1/2 u_a div u exactly (up to rounding).  A
  wrong averaging index, a dropped half, a sign or a transposed component
  breaks it.
- Skew symmetry.  On a periodic grid the central difference is
  antisymmetric, so for every component a and any velocity,
  sum over the a-faces of u_a N_a(u) vanishes (summation by parts cancels
  the two halves).  Dropping or rescaling one half, or a one-sided
  difference, breaks it.
- Boundary rows.  For a smooth velocity meeting the boundary conditions
  (no-slip walls, prescribed inflow, zero normal derivative at the outflow),
  N_a converges to the continuum term at second order at every unknown face,
  boundary rows included: a wrong ghost rule shows up as an error that does
  not fall with h.
"""
import numpy as np
import pytest
import sympy as sp

import oracle as O
from paper_1302_3663_amd import synth

import mms_fields as M


def advection(p, u):
    nf = sum(O.face_counts(p))
    rho = np.ones(nf)
    mc = np.ones(O.cell_count(p))
    me = np.ones(sum(O.edge_counts(p)))
    b = O.momentum_rhs(p, u, rho, mc, me, np.zeros(nf), with_boundary=False)
    return p["sigma"] / p["dt"] * u - b


def unknown_rows(p):
    nf = sum(O.face_counts(p))
    H = O.Hierarchy(p, np.ones(nf), np.ones(O.cell_count(p)), np.ones(sum(O.edge_counts(p))))
    return H.unknowns(True)


GRIDS = {
    "2d_inout": lambda: synth.base_params(2, [14, 12], [O.AX_INOUT, O.AX_WALLS], 1.0 / 12),
    "2d_channel": lambda: synth.base_params(2, [14, 12], [O.AX_PERIODIC, O.AX_WALLS], 1.0 / 12),
    "3d_tube": lambda: synth.base_params(3, [10, 12, 14], [O.AX_WALLS, O.AX_WALLS, O.AX_INOUT], 1.0 / 10),
}


@pytest.mark.parametrize("g", sorted(GRIDS))
def test_advection_exact_for_linear_velocity(g):
    p = GRIDS[g]()
    D = p["dim"]
    rng = np.random.default_rng(7)
    G = rng.standard_normal((D, D))       # u_b(x) = c_b + G[b] . x
    c = rng.standard_normal(D)
    u = np.concatenate([c[a] + M.all_points(p, O.FACE, a) @ G[a] for a in range(D)])
    N = O.split_faces(p, advection(p, u))
    comp, pos = unknown_rows(p)
    checked = 0
    for a in range(D):
        q = pos[comp == a]
        # every position the stencil reads is stored: two away from each end
        ok = np.ones(q.shape[0], bool)
        for d in range(D):
            ok &= (q[:, d] >= 2) & (q[:, d] <= p["n"][d] - 3)
        q = q[ok]
        x = M.coords_of(p, O.FACE, a, q)
        ub = c[None, :] + x @ G.T              # u at these faces, all components
        want = np.einsum("nb,b->n", ub, G[a]) + 0.5 * ub[:, a] * np.trace(G)
        got = N[a][q[:, 2], q[:, 1], q[:, 0]]
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())
        checked += q.shape[0]
    assert checked > 50


@pytest.mark.parametrize("dim", [2, 3])
def test_advection_skew_symmetric_on_periodic_grid(dim):
    n = [12, 10] if dim == 2 else [8, 10, 12]
    p = synth.base_params(dim, n, [O.AX_PERIODIC] * dim, 1.0 / 10)
    rng = np.random.default_rng(8)
    u = rng.standard_normal(sum(O.face_counts(p)))
    N = advection(p, u)
    uf, Nf = O.split_faces(p, u), O.split_faces(p, N)
    for a in range(dim):
        s = np.sum(uf[a] * Nf[a])
        scale = np.sum(np.abs(uf[a] * Nf[a]))
        assert abs(s) <= 1e-13 * scale, (a, s, scale)
        assert scale > 1.0


def _velocity_2d(Lx, bcx):
    x, y = M.X, M.Y
    S, C, pi = sp.sin, sp.cos, sp.pi
    if bcx == O.AX_INOUT:     # inflow at x = 0 (u_y odd there), outflow at x = Lx (even)
        xt, xn = S(pi * x / (2 * Lx)), 1 + C(pi * (x - Lx) / Lx) / 2
    else:
        xt, xn = S(2 * pi * x / Lx) + sp.Rational(1, 2), C(2 * pi * x / Lx) + 1
    ux = S(pi * y) * (1 + C(pi * y) / 3) * xn
    uy = S(pi * y) * (1 + C(2 * pi * y) / 2) * xt
    return [ux, uy]


def _velocity_3d(Lz):
    x, y, z = M.X, M.Y, M.Z
    S, C, pi = sp.sin, sp.cos, sp.pi
    zt = S(pi * z / (2 * Lz))      # odd about the inflow plane, even about the outflow
    ux = S(pi * x) * (1 + C(2 * pi * x) / 2) * S(pi * y) * zt
    uy = S(pi * y) * S(2 * pi * x) * (1 + C(pi * y) / 3) * zt
    uz = S(pi * x) * S(pi * y) * (1 + C(pi * (z - Lz) / Lz) / 2)
    return [ux, uy, uz]


def _max_error(p, u_exprs):
    D = p["dim"]
    N_exact = [sum(u_exprs[b] * sp.diff(u_exprs[a], M.SYMS[b]) for b in range(D))
               + u_exprs[a] * sum(sp.diff(u_exprs[b], M.SYMS[b]) for b in range(D)) / 2 for a in range(D)]
    N = advection(p, M.faces(p, u_exprs))
    comp, pos = unknown_rows(p)
    got = M.gather(p, N, comp, pos)
    want = np.zeros_like(got)
    for a in range(D):
        s = comp == a
        want[s] = M.evaluate(N_exact[a], M.coords_of(p, O.FACE, a, pos[s]))
    return np.abs(got - want).max() / np.abs(want).max()


@pytest.mark.parametrize("case", ["2d_inout", "2d_channel", "3d_tube"])
def test_advection_second_order_at_every_row(case):
    errs = []
    sizes = (16, 32, 64) if case != "3d_tube" else (16, 32, 64)
    for n in sizes:
        h = 1.0 / n
        if case == "3d_tube":
            p = synth.base_params(3, [n, n, n], [O.AX_WALLS, O.AX_WALLS, O.AX_INOUT], h)
            u = _velocity_3d(1.0)
        else:
            bcx = O.AX_INOUT if case == "2d_inout" else O.AX_PERIODIC
            p = synth.base_params(2, [2 * n, n], [bcx, O.AX_WALLS], h)
            u = _velocity_2d(2.0, bcx)
        errs.append(_max_error(p, u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.diff(errs) < 0), errs
    assert rates[-1] > 1.85, (errs, rates)
