"""Pins for the immersed-boundary transfers (eq:discrForceCouple,
eq:discrDensCouple, eq:discrVelCouple, eq:ViscExp).

- spread and interpolation with equal widths are adjoint:
  <S F, u>_{h^D} = <F, J u> (each sums delta~ over the same closed-domain
  points, so the identity is exact up to rounding);
- the support enumeration matches a brute-force sum over every lattice point;
- with width h the unity condition holds exactly, so J reproduces constants
  and the spread integral equals the total node quantity;
- the viscosity field is a max (not a sum): mu = mu_max at a node on a
  lattice point, mu_out <= mu <= mu_max, mu_out outside every support;
- the worked-example inputs of Fig. ForceEx / Fig. ViscEx (tests/golden).
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1302_3663_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def lattice_points(p, kind, axis):
    """coordinates of every closed-domain point of a lattice, compact order"""
    n, dims = O.lattice_dims(p, kind, axis)
    h = p["h"]
    axes = []
    for d in range(3):
        if d >= p["dim"]:
            axes.append(np.zeros(1))
            continue
        vert = (kind == O.FACE and d == axis) or (kind == O.EDGE and d != axis)
        q = np.arange(dims[d])
        axes.append(q * h if vert else (q + 0.5) * h)
    Z, Y, Xc = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([Xc.ravel(), Y.ravel(), Z.ravel()])[:p["dim"]]


def brute_delta(p, pts, X, width, kernel=0):
    """delta~(x - X, w) for every (point, node) pair, nearest image on periodic axes"""
    W = np.ones((pts.shape[1], X.shape[1])) / width ** p["dim"]
    for d in range(p["dim"]):
        diff = pts[d][:, None] - X[d][None, :]
        if p["axis_bc"][d] == O.AX_PERIODIC:
            Lx = p["n"][d] * p["h"]
            diff = diff - Lx * np.round(diff / Lx)
        W *= O.phi(kernel, (diff / width).ravel()).reshape(diff.shape)
    return W


CASES = {
    "2d_periodic_walls": lambda: synth.tiny_2d(),
    "2d_inout_walls": lambda: synth.tiny_2d(inout=True),
    "3d_tube": lambda: synth.tiny_3d(),
    "3d_periodic_z": lambda: synth.tiny_3d(periodic_z=True),
}


def nodes_near_boundaries(p, rng, eta):
    """random nodes including some across a periodic seam and next to walls"""
    Lx = [p["n"][d] * p["h"] for d in range(p["dim"])]
    X = np.stack([rng.uniform(0, Lx[d], eta) for d in range(p["dim"])])
    X[:, 0] = [0.01 * Lx[d] for d in range(p["dim"])]
    X[:, 1] = [0.995 * Lx[d] for d in range(p["dim"])]
    return X


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("wsel", ["omega", "h"])
def test_spread_interp_adjoint(case, wsel):
    c = CASES[case]()
    p = c["params"]
    w = p["omega"] if wsel == "omega" else p["h"]
    rng = np.random.default_rng(5)
    X = nodes_near_boundaries(p, rng, 17)
    F = rng.standard_normal(X.shape)
    u = rng.standard_normal(sum(O.face_counts(p)))
    SF = O.spread_vec(p, w, X, F)
    JU = O.interp_vec(p, w, X, u)
    lhs = (SF * u).sum() * p["h"] ** p["dim"]
    rhs = (F * JU).sum()
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.abs(F * JU).sum())


@pytest.mark.parametrize("case", sorted(CASES))
def test_spread_matches_brute_force(case):
    c = CASES[case]()
    p = c["params"]
    rng = np.random.default_rng(6)
    X = nodes_near_boundaries(p, rng, 9)
    F = rng.standard_normal(X.shape)
    got = O.split_faces(p, O.spread_vec(p, p["omega"], X, F))
    for a in range(p["dim"]):
        pts = lattice_points(p, O.FACE, a)
        W = brute_delta(p, pts, X, p["omega"])
        want = W @ F[a]
        np.testing.assert_allclose(got[a].ravel(), want, rtol=1e-13, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("case", sorted(CASES))
def test_viscosity_matches_brute_force_max(case):
    c = CASES[case]()
    p = c["params"]
    X = c["X"]
    mc = O.viscosity_cells(p, X)
    W = brute_delta(p, lattice_points(p, O.CELL, 0), X, p["omega"])
    want = np.maximum(p["mu_out"], ((2 * p["omega"]) ** p["dim"] * (p["mu_max"] - p["mu_out"]) * W
                                    + p["mu_out"]).max(axis=1))
    np.testing.assert_allclose(mc, want, rtol=1e-14)
    me = O.viscosity_edges(p, X)
    axes = [0, 1, 2] if p["dim"] == 3 else [2]
    off = 0
    for ax in axes:
        pts = lattice_points(p, O.EDGE, ax)
        W = brute_delta(p, pts, X, p["omega"])
        want = np.maximum(p["mu_out"], ((2 * p["omega"]) ** p["dim"] * (p["mu_max"] - p["mu_out"]) * W
                                        + p["mu_out"]).max(axis=1))
        np.testing.assert_allclose(me[off:off + pts.shape[1]], want, rtol=1e-14)
        off += pts.shape[1]


def test_viscosity_is_max_not_sum():
    c = synth.tiny_2d()
    p = c["params"]
    h = p["h"]
    X = np.array([[7.5 * h], [4.5 * h]])             # the centre of cell (7, 4)
    one = O.viscosity_cells(p, X)
    two = O.viscosity_cells(p, np.concatenate([X, X], axis=1))
    np.testing.assert_array_equal(one, two)
    # the node sits on the centre of cell (7, 4): mu = mu_max there exactly
    assert abs(one.reshape(p["n"][1], p["n"][0])[4, 7] - p["mu_max"]) < 1e-12
    assert one.min() >= p["mu_out"] and one.max() <= p["mu_max"] * (1 + 1e-15)
    far = one.reshape(p["n"][1], p["n"][0])[:, 0]
    assert np.all(far == p["mu_out"])


def test_unity_with_width_h_interior():
    # delta~ with width h satisfies the unity condition exactly: J reproduces a
    # constant and the spread integral equals the node total
    c = synth.tiny_3d(periodic_z=True)
    p = c["params"]
    rng = np.random.default_rng(7)
    X = np.stack([rng.uniform(0.3, 0.7, 6), rng.uniform(0.3, 0.7, 6), rng.uniform(0, 2, 6)])
    u = np.full(sum(O.face_counts(p)), 1.7)
    U = O.interp_vec(p, p["h"], X, u)
    np.testing.assert_allclose(U, 1.7, rtol=1e-14)
    F = rng.standard_normal(X.shape)
    S = O.split_faces(p, O.spread_vec(p, p["h"], X, F))
    for a in range(3):
        assert abs(S[a].sum() * p["h"] ** 3 - F[a].sum()) < 1e-13 * np.abs(F[a]).sum()


def test_density_integral_width_h():
    c = synth.tiny_3d(periodic_z=True)
    p = dict(c["params"])
    p["omega"] = p["h"]
    rng = np.random.default_rng(8)
    X = np.stack([rng.uniform(0.3, 0.7, 5), rng.uniform(0.3, 0.7, 5), rng.uniform(0, 2, 5)])
    rho = O.split_faces(p, O.density(p, X))
    for a in range(3):
        tot = (rho[a] - p["rho0"]).sum() * p["h"] ** 3
        assert abs(tot - p["rho_b"] * p["d0_pow_d"] * X.shape[1]) < 1e-13


def test_worked_example_force_and_viscosity():
    """Fig. ForceEx / Fig. ViscEx inputs embedded in 2D with every node on the
    line y = (j + 1/2) h: the force spread integral is the sum of node forces
    (zero here) up to the unity defect, and mu hits mu_max at the node that
    sits on a lattice point."""
    g = json.load(open(os.path.join(GOLD, "worked_example_fig_forceex.json")))
    omega = g["omega"]
    for h in g["h"]:
        n = int(round(1.0 / h))
        p = synth.base_params(2, [n, n], [O.AX_PERIODIC, O.AX_WALLS], h)
        p.update(omega=omega, mu_out=1.0, mu_max=5.0)
        y0 = (n // 2 + 0.5) * h
        X = np.array([g["X"], [y0] * 3])
        F = np.array([g["F"], [0.0] * 3])
        S = O.split_faces(p, O.spread_vec(p, omega, X, F))
        integral = S[0].sum() * h * h
        # the unity defect of delta~ bounds the integral: |sum F_s e_s|
        pts = lattice_points(p, O.FACE, 0)
        W = brute_delta(p, pts, X, omega)
        e = W.sum(axis=0) * h * h - 1.0
        assert abs(integral - (F[0] * (1 + e)).sum()) < 1e-12
        assert abs(sum(g["F"])) == 0.0
        mu = O.viscosity_cells(p, X[:, :2]).reshape(n, n)
        # first node x = 5/32 is a face position; the cell-centred mu peaks
        # next to it and never exceeds mu_max
        assert mu.max() <= p["mu_max"] * (1 + 1e-15)
        assert mu.min() >= p["mu_out"]
