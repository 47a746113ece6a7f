"""Pins of the oracle's constant-viscosity momentum operator (eq:NSdis1):
(sigma rho / dt) u_a - Re^-1 mu L_h u_a, one independent system per
component.  What fixes it, independently of the oracle's stencil code:
- Fourier modes on a fully periodic grid are eigenvectors with the closed-form
  eigenvalue of the discrete Laplacian, on the finest level and on a coarse
  level whose viscosity carries gamma;
- the coupled operator of eq:NSdis1-1 at the same constant viscosity differs
  from it by exactly -Re^-1 mu D_a(div u), the term the paper drops by
  incompressibility (div and its gradient computed here on the MAC lattice);
- with walls and inflow/outflow it equals a Kronecker sum of 1D second
  differences built here from the boundary readings (odd tangential images at
  walls and the inflow, even images at the outflow, Dirichlet wall-normal
  faces);
- the multigrid solve of it converges to the sparse direct solution;
- the form is refused when the viscosity is not one constant."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_1302_3663_amd import synth

P_, W_, IO_ = O.AX_PERIODIC, O.AX_WALLS, O.AX_INOUT


def params(dim, n, bc, mu=2.5, gamma1=0.7, decoupled=1):
    p = synth.base_params(dim, list(n), list(bc), 1.0 / n[0])
    p.update(mu_out=mu, mu_max=mu, decoupled=decoupled)
    p["gamma"] = [1.0, gamma1] + [1.0] * 14
    return p


def hierarchy(p, rho=1.3, rng=None):
    nf = sum(O.face_counts(p))
    r = np.full(nf, rho) if rng is None else rho * (1.0 + 0.2 * rng.random(nf))
    mc = np.full(O.cell_count(p), p["mu_out"])
    me = np.full(sum(O.edge_counts(p)), p["mu_out"])
    return O.Hierarchy(p, r, mc, me)


def eig(p, level, theta, rho):
    h = p["h"] * 2 ** level
    mu = p["mu_out"] * (p["gamma"][1] if level >= 1 else 1.0)
    lap = sum(4.0 * math.sin(t / 2) ** 2 for t in theta) / (h * h)
    return p["sigma"] / p["dt"] * rho + p["inv_re"] * mu * lap


@pytest.mark.parametrize("dim,n", [(2, (16, 8)), (3, (8, 8, 4))])
@pytest.mark.parametrize("level", [0, 1])
def test_fourier_modes_are_eigenvectors(dim, n, level):
    p = params(dim, n, [P_] * dim)
    H = hierarchy(p)
    comp, pos = H.unknowns(True, level)
    dims = H.dims[level]
    rng = np.random.default_rng(3)
    for a in range(dim):
        k = rng.integers(1, 4, size=3)
        theta = [2 * math.pi * k[b] / dims[b] for b in range(dim)]
        x = np.zeros(len(comp))
        sel = comp == a
        x[sel] = np.cos(sum(theta[b] * pos[sel, b] for b in range(dim)) + 0.3)
        y = H.apply_vec(True, x, level)
        lam = eig(p, level, theta, 1.3)
        assert np.max(np.abs(y - lam * x)) <= 1e-12 * lam


def mac_div_grad(p, comp, pos, u):
    """-> D_a(div u) at every velocity unknown of a fully periodic grid."""
    dim, n, h = p["dim"], p["n"], p["h"]
    shape = tuple(n[b] for b in range(dim))
    U = [np.zeros(shape) for _ in range(dim)]
    for a in range(dim):
        s = comp == a
        U[a][tuple(pos[s, b] for b in range(dim))] = u[s]
    # the high face of cell q along b is face q + e_b
    div = sum((np.roll(U[b], -1, axis=b) - U[b]) / h for b in range(dim))
    out = np.zeros_like(u)
    for a in range(dim):
        s = comp == a
        g = (div - np.roll(div, 1, axis=a)) / h   # face q lies between cells q - e_a and q
        out[s] = g[tuple(pos[s, b] for b in range(dim))]
    return out


@pytest.mark.parametrize("dim,n", [(2, (16, 8)), (3, (8, 8, 4))])
def test_coupled_minus_decoupled_is_grad_div(dim, n):
    pd = params(dim, n, [P_] * dim, decoupled=1)
    pc = params(dim, n, [P_] * dim, decoupled=0)
    rng = np.random.default_rng(5)
    Hd, Hc = hierarchy(pd, rng=np.random.default_rng(9)), hierarchy(pc, rng=np.random.default_rng(9))
    comp, pos = Hd.unknowns(True)
    u = rng.standard_normal(len(comp))
    diff = Hc.apply_vec(True, u) - Hd.apply_vec(True, u)
    want = -pd["inv_re"] * pd["mu_out"] * mac_div_grad(pd, comp, pos, u)
    scale = np.max(np.abs(Hc.apply_vec(True, u)))
    assert np.max(np.abs(diff - want)) <= 1e-12 * scale
    assert np.max(np.abs(want)) > 1e-3 * scale   # the dropped term is not negligible here
    # a discretely divergence-free field (curl of a stream function) sees no difference
    if dim == 2:
        nx, ny = n
        psi = rng.standard_normal((ny, nx))        # at cell corners (i, j)
        h = pd["h"]
        ux = (np.roll(psi, -1, axis=0) - psi) / h  # d psi / dy at x-faces
        uy = -(np.roll(psi, -1, axis=1) - psi) / h
        v = np.zeros(len(comp))
        for a, F in ((0, ux), (1, uy)):
            s = comp == a
            v[s] = F[pos[s, 1], pos[s, 0]]
        assert np.max(np.abs(mac_div_grad(pd, comp, pos, v))) <= 1e-9 * np.max(np.abs(v)) / h ** 2
        d2 = Hc.apply_vec(True, v) - Hd.apply_vec(True, v)
        assert np.max(np.abs(d2)) <= 1e-12 * np.max(np.abs(Hc.apply_vec(True, v)))


def second_difference(kind, bc, n):
    """1D second difference (unit spacing) on the unknowns of one axis.
    kind 'v': the component's own axis (faces), 'c': another axis (cells)."""
    if kind == "v":
        m = n if bc in (P_, IO_) else n - 1
    else:
        m = n
    T = np.zeros((m, m))
    for i in range(m):
        T[i, i] = -2.0
        if i > 0:
            T[i, i - 1] = 1.0
        if i < m - 1:
            T[i, i + 1] = 1.0
    if bc == P_:
        T[0, m - 1] += 1.0
        T[m - 1, 0] += 1.0
    elif kind == "v" and bc == IO_:
        T[m - 1, m - 2] += 1.0      # outflow face: the outside image mirrors the face below it
    elif kind == "c":
        T[0, 0] -= 1.0              # odd image at the wall / inflow
        T[m - 1, m - 1] += -1.0 if bc == W_ else 1.0   # odd at a wall, even at the outflow
    return T


def lo_index(kind, bc):
    return 1 if (kind == "v" and bc != P_) else 0


@pytest.mark.parametrize("dim,n,bc", [
    (2, (16, 8), (P_, W_)),
    (2, (16, 8), (IO_, W_)),
    (3, (8, 8, 16), (W_, W_, IO_)),
    (3, (8, 8, 8), (W_, W_, P_)),
])
def test_equals_kronecker_sum_with_boundaries(dim, n, bc):
    p = params(dim, n, bc)
    H = hierarchy(p)
    comp, pos = H.unknowns(True)
    A = H.csr(True)
    # no coupling between components
    r, c = A.nonzero()
    assert np.all(comp[r] == comp[c])
    rng = np.random.default_rng(2)
    x = rng.standard_normal(len(comp))
    y = A @ x
    h = p["h"]
    for a in range(dim):
        s = comp == a
        kinds = ["v" if b == a else "c" for b in range(dim)]
        Ts = [second_difference(kinds[b], bc[b], n[b]) for b in range(dim)]
        shape = tuple(T.shape[0] for T in Ts)
        idx = tuple(pos[s, b] - lo_index(kinds[b], bc[b]) for b in range(dim))
        X = np.zeros(shape)
        X[idx] = x[s]
        assert np.count_nonzero(s) == X.size
        lap = sum(np.moveaxis(np.tensordot(Ts[b], X, axes=([1], [b])), 0, b) for b in range(dim)) / (h * h)
        Y = p["sigma"] / p["dt"] * 1.3 * X - p["inv_re"] * p["mu_out"] * lap
        assert np.max(np.abs(Y[idx] - y[s])) <= 1e-12 * np.max(np.abs(Y))


def to_unknowns(H, p, compact):
    comp, pos = H.unknowns(True)
    faces = O.split_faces(p, compact)
    return np.array([faces[a][k, j, i] for a, (i, j, k) in zip(comp, pos)])


@pytest.mark.parametrize("dim,n,bc", [(2, (16, 8), (IO_, W_)), (3, (8, 8, 16), (W_, W_, IO_))])
def test_solve_matches_direct(dim, n, bc):
    p = params(dim, n, bc)
    p["rtol"] = 1e-11
    H = hierarchy(p, rng=np.random.default_rng(4))
    comp, _ = H.unknowns(True)
    rng = np.random.default_rng(6)
    nf = sum(O.face_counts(p))
    b = rng.standard_normal(nf)
    x, info = H.solve(True, b, np.zeros(nf))
    assert info["status"] == 0 and info["relres"] <= p["rtol"]
    assert H.relres(True, b, x) <= p["rtol"] * (1 + 1e-6)
    A = H.csr(True)
    bu, xu = to_unknowns(H, p, b), to_unknowns(H, p, x)
    xs = spla.spsolve(A.tocsc(), bu)
    assert np.linalg.norm(xu - xs) <= 1e-9 * np.linalg.norm(xs)


def test_refused_with_variable_viscosity():
    p = params(2, (16, 8), (P_, W_))
    p["mu_max"] = 3.0
    with pytest.raises(Exception):
        hierarchy(p)


def test_steps_stay_close_to_the_coupled_form():
    """The two forms differ by Re^-1 mu D_a(div u~), and u~ is divergence-free
    only up to the projection's correction, so whole steps of the two agree
    closely but not to rounding."""
    from oracle import step as S
    base = synth.tiny_2d()
    out = []
    for dec in (0, 1):
        p = dict(base["params"], decoupled=dec)
        p["mu_max"] = p["mu_out"]
        st = S.State(p, base["u0"], base["p0"], base["X"], base["ij"], base["rest"], base["K"])
        S.setup(st)
        for _ in range(3):
            S.projection_step(st)
            S.lagrangian_update(st)
        out.append(st.u.copy())
    d = np.linalg.norm(out[1] - out[0]) / np.linalg.norm(out[0])
    assert 1e-12 < d < 1e-4
