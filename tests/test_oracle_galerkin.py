"""Pins for the Galerkin coarse operators of the viscous system (the second
remedy that Sec. "Numerical Concerns" names for slow convergence at large
mu_max: coarse operators that satisfy the Galerkin condition).

- every coarse matrix equals the dense product R A P, with R and P built
  column by column from the oracle's own restriction and prolongation
  (pinned in test_oracle_mg) and A the next finer matrix;
- the pressure matrices and the finest viscous matrix do not change;
- Galerkin condition: a two-level correction with an exact coarse solve
  leaves a fine residual whose restriction vanishes (rediscretised coarse
  operators do not have this property, which the test also shows);
- the smoother of a Galerkin level (a red-black sweep, Jacobi inside each
  (component, colour) set because R A P couples points of one colour) keeps
  the exact solution fixed, equals that set-by-set rule written with dense
  matrices, and equals plain Gauss-Seidel wherever no two rows of a set
  couple (the rediscretised levels);
- at a viscosity ratio of 1e3 the V-cycles need fewer cycles to the
  tolerance than with rediscretised coarse operators.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_1302_3663_amd import synth


CASES = {
    "2d_periodic_walls": lambda: synth.tiny_2d(),
    "2d_inout_walls": lambda: synth.tiny_2d(inout=True),
    "3d_tube": lambda: synth.tiny_3d(),
    "3d_periodic_z": lambda: synth.tiny_3d(periodic_z=True),
    "channel2d_64x32": lambda: synth.channel_2d(seed=1),
}


def hierarchy(case, **over):
    p = dict(case["params"], **over)
    X = case["X"]
    return O.Hierarchy(p, O.density(p, X), O.viscosity_cells(p, X), O.viscosity_edges(p, X)), p


def dense_transfers(H, l):
    nf, nc = H.csr(True, l).shape[0], H.csr(True, l + 1).shape[0]
    P = np.array([H.prolong_vec(True, l, np.eye(1, nc, j).ravel()) for j in range(nc)]).T
    R = np.array([H.restrict_vec(True, l, np.eye(1, nf, j).ravel()) for j in range(nf)]).T
    return R, P


def to_unknowns(H, p, compact):
    comp, pos = H.unknowns(True, 0)
    faces = O.split_faces(p, compact)
    return np.array([faces[a][k, j, i] for a, (i, j, k) in zip(comp, pos)])


@pytest.mark.parametrize("name", sorted(CASES))
def test_coarse_matrices_are_dense_rap(name):
    case = CASES[name]()
    H, _ = hierarchy(case, galerkin=1)
    Hr, _ = hierarchy(case, galerkin=0)
    assert H.levels >= 2
    for l in range(1, H.levels):
        A = H.csr(True, l - 1).toarray()
        R, P = dense_transfers(H, l - 1)
        G = H.csr(True, l).toarray()
        ref = R @ A @ P
        assert np.abs(G - ref).max() <= 1e-13 * np.abs(ref).max(), l
        # a wider stencil than the rediscretised operator's
        assert H.csr(True, l).nnz > Hr.csr(True, l).nnz
    # the rest of the hierarchy is untouched
    assert (H.csr(True, 0) != Hr.csr(True, 0)).nnz == 0
    for l in range(H.levels):
        assert (H.csr(False, l) != Hr.csr(False, l)).nnz == 0


@pytest.mark.parametrize("name", ["2d_periodic_walls", "2d_inout_walls"])
def test_two_level_correction_annihilates_restricted_residual(name):
    """R (b - A (x + P G^-1 R (b - A x))) = 0 exactly when G = R A P; the
    oracle's own V-cycle (no smoothing, two levels, dense coarse solve)
    performs that correction."""
    case = CASES[name]()
    rng = np.random.default_rng(5)
    ratios = {}
    for gal in (1, 0):
        H, p = hierarchy(case, galerkin=gal, nu1=0, nu2=0, max_levels=2)
        assert H.levels == 2 and H.csr(True, 1).shape[0] <= 64   # coarse level solved densely
        A = H.csr(True, 0)
        nb = int(sum(O.face_counts(p)))
        b = rng.standard_normal(nb)
        x0 = np.zeros(nb)
        x1 = H.vcycles(True, b, x0, 1)
        bu = to_unknowns(H, p, b)
        r0 = bu - A @ to_unknowns(H, p, x0)
        r1 = bu - A @ to_unknowns(H, p, x1)
        ratios[gal] = np.linalg.norm(H.restrict_vec(True, 0, r1)) / np.linalg.norm(H.restrict_vec(True, 0, r0))
    assert ratios[1] < 1e-12
    assert ratios[0] > 1e-3


def set_sweep(G, comp, pos, b, x):
    """One sweep by (component, colour) sets: x_S += D_S^-1 (b - G x)_S."""
    x = x.copy()
    colour = pos.sum(axis=1) % 2
    d = G.diagonal()
    for c in range(int(comp.max()) + 1):
        for k in range(2):
            S = np.nonzero((comp == c) & (colour == k))[0]
            r = b[S] - G[S] @ x
            x[S] = x[S] + r / d[S]
    return x


@pytest.mark.parametrize("name", sorted(CASES))
def test_galerkin_level_smoother(name):
    case = CASES[name]()
    H, _ = hierarchy(case, galerkin=1)
    Hr, _ = hierarchy(case, galerkin=0)
    rng = np.random.default_rng(6)
    for l in range(1, H.levels):
        G = H.csr(True, l).tocsr()
        comp, pos = H.unknowns(True, l)
        n = G.shape[0]
        b = rng.standard_normal(n)
        # the exact solution is a fixed point
        xs = spla.spsolve(G.tocsc(), b)
        assert np.abs(H.smooth_level(True, l, b, xs, 1) - xs).max() <= 1e-12 * np.abs(xs).max()
        # the sweep is the set-by-set rule
        x0 = rng.standard_normal(n)
        got = H.smooth_level(True, l, b, x0, 2)
        ref = set_sweep(G, comp, pos, b, set_sweep(G, comp, pos, b, x0))
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        # where no two rows of a set couple, the same rule is Gauss-Seidel:
        # on the rediscretised level the oracle's sequential sweep agrees
        Gr = Hr.csr(True, l).tocsr()
        got_r = Hr.smooth_level(True, l, b, x0, 1)
        assert np.abs(got_r - set_sweep(Gr, comp, pos, b, x0)).max() <= 1e-12 * np.abs(got_r).max()


@pytest.mark.parametrize("name", ["3d_tube", "channel2d_64x32"])
def test_fewer_cycles_than_rediscretised(name):
    case = CASES[name]()
    cycles = {}
    for gal in (0, 1):
        H, p = hierarchy(case, galerkin=gal, gamma=[1.0] * 16)
        nb = int(sum(O.face_counts(p)))
        b = np.random.default_rng(7).standard_normal(nb)
        x, info = H.solve(True, b, np.zeros(nb))
        assert info["relres"] <= p["rtol"]
        cycles[gal] = info["cycles"]
    assert cycles[1] < cycles[0], cycles


def test_fewer_cycles_at_viscosity_ratio_1e3():
    """16x16x32 tube with mu_max / mu_out = 1e3: Galerkin coarse operators
    reach the tolerance in clearly fewer V-cycles (16 against 23 when this
    test was written)."""
    case = synth.tube_3d(seed=3, n=(16, 16, 32), eta=800, spacing=0.04, cutoff=0.1, rho_b=0.2, mu_max=1e3,
                         omega=0.04)
    cycles = {}
    for gal in (0, 1):
        H, p = hierarchy(case, galerkin=gal, gamma=[1.0] * 16)
        nb = int(sum(O.face_counts(p)))
        b = np.random.default_rng(0).standard_normal(nb)
        _, info = H.solve(True, b, np.zeros(nb))
        assert info["relres"] <= p["rtol"]
        cycles[gal] = info["cycles"]
    assert cycles[1] <= 0.8 * cycles[0], cycles


def test_flag_checks():
    case = synth.tiny_2d()
    for over in (dict(galerkin=2), dict(galerkin=1, decoupled=1, mu_max=case["params"]["mu_out"])):
        with pytest.raises(RuntimeError):
            hierarchy(case, **over)
