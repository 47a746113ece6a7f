"""Pins for the multigrid solver (Sec. "Multigrid", eq:resCondrelationship,
the work-unit study of Fig. "Work Units Decrease 2D").

- the probe-assembled matrix equals column-by-column application of the
  stencil to unit vectors (brute force);
- the matrices are symmetric and positive definite except where the outflow
  face sits (its row uses a one-sided mirror), and the all-Neumann/periodic
  pressure matrix has exactly the constants as null space;
- restriction is 2^-D times the transpose of prolongation (full weighting
  against linear interpolation) away from outflow faces;
- constant-coefficient systems reduce to library transforms: the periodic x
  Neumann-y pressure Laplacian is diagonalised by an FFT in x and a DCT-II in
  y, and the doubly and triply periodic MAC viscous operator by an FFT whose
  symbol per wavenumber k is sigma rho/dt I + Re^-1 mu (|s|^2 I + s s^T),
  s_d = 2 sin(k_d h / 2) / h;
- V-cycle solves agree with a sparse direct solve within cond * rtol;
- adding levels cuts the work units to reach the tolerance by orders of
  magnitude (1 level is plain relaxation);
- the condition number grows like h^-2.
"""
import numpy as np
import pytest
import scipy.fft as sfft
import scipy.sparse.linalg as spla

import oracle as O
from paper_1302_3663_amd import synth


def coefs_of(case):
    p = case["params"]
    X = case["X"]
    return O.density(p, X), O.viscosity_cells(p, X), O.viscosity_edges(p, X)


CASES = {
    "2d_periodic_walls": lambda: synth.tiny_2d(),
    "2d_inout_walls": lambda: synth.tiny_2d(inout=True),
    "3d_tube": lambda: synth.tiny_3d(),
    "3d_periodic_z": lambda: synth.tiny_3d(periodic_z=True),
}


def hier(case):
    c = CASES[case]()
    return c, O.Hierarchy(c["params"], *coefs_of(c))


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("vel", [False, True])
def test_probe_assembly_equals_brute_force(case, vel):
    c, H = hier(case)
    for level in range(H.levels):
        A = H.csr(vel, level).toarray()
        n = A.shape[0]
        B = np.zeros_like(A)
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            B[:, j] = H.apply_vec(vel, e, level)
        np.testing.assert_array_equal(A, B)


@pytest.mark.parametrize("case", sorted(CASES))
def test_symmetry_definiteness_nullspace(case):
    c, H = hier(case)
    p = c["params"]
    inout = any(p["axis_bc"][a] == O.AX_INOUT for a in range(p["dim"]))
    for vel in (False, True):
        A = H.csr(vel).toarray()
        asym = np.abs(A - A.T).max() / np.abs(A).max()
        if vel and inout:
            assert asym > 0      # the outflow row mirrors one-sidedly
            ev = np.linalg.eigvals(A)
            assert ev.real.min() > 0
            continue
        assert asym < 1e-15
        ev = np.linalg.eigvalsh(A)
        if not vel and not inout:
            # singular: exactly one zero eigenvalue with the constants as null vector
            assert abs(ev[0]) < 1e-10 * ev[-1] and ev[1] > 1e-6 * ev[-1]
            assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-10 * ev[-1]
        else:
            assert ev[0] > 0


@pytest.mark.parametrize("case", ["2d_periodic_walls", "3d_periodic_z"])
@pytest.mark.parametrize("vel", [False, True])
def test_restriction_is_scaled_transpose_of_prolongation(case, vel):
    c, H = hier(case)
    D = c["params"]["dim"]
    for level in range(H.levels - 1):
        nf = H.nunk[level][1 if vel else 0]
        nc = H.nunk[level + 1][1 if vel else 0]
        R = np.stack([H.restrict_vec(vel, level, e) for e in np.eye(nf)], axis=1)
        Pm = np.stack([H.prolong_vec(vel, level, e) for e in np.eye(nc)], axis=1)
        np.testing.assert_allclose(R, Pm.T / 2 ** D, atol=1e-16)
        # constants are prolonged exactly in the interior of periodic axes
        assert np.all(np.abs(Pm.sum(axis=1)) <= 1.0 + 1e-15)


def test_pressure_matches_fft_dct():
    nx, ny = 32, 16
    p = synth.base_params(2, [nx, ny], [O.AX_PERIODIC, O.AX_WALLS], 1.0 / ny)
    H = O.Hierarchy(p, np.ones(sum(O.face_counts(p))), np.ones(O.cell_count(p)), np.ones(sum(O.edge_counts(p))))
    rng = np.random.default_rng(4)
    b = rng.standard_normal((ny, nx))
    b -= b.mean()
    x, st = H.solve(False, b.ravel(), np.zeros(nx * ny))
    assert st["status"] == 0 and st["relres"] <= 1e-10
    h = p["h"]
    bh = sfft.dct(np.fft.fft(b, axis=1), type=2, norm="ortho", axis=0)
    m = np.arange(nx)
    k = np.arange(ny)
    lam = (4 / h ** 2) * (np.sin(np.pi * m / nx)[None, :] ** 2 + np.sin(np.pi * k / (2 * ny))[:, None] ** 2)
    lam[0, 0] = 1.0
    ph = bh / lam
    ph[0, 0] = 0.0
    pe = np.real(np.fft.ifft(sfft.idct(ph, type=2, norm="ortho", axis=0), axis=1))
    xs = x.reshape(ny, nx) - x.mean()
    cond = lam.max() / lam[lam > 1e-9].min()
    assert np.linalg.norm(xs - pe) <= cond * 1e-10 * np.linalg.norm(pe)
    assert np.linalg.norm(xs - pe) <= 1e-8 * np.linalg.norm(pe)


@pytest.mark.parametrize("dims", [(16, 8), (8, 8, 8)])
def test_viscous_matches_fourier_symbol(dims):
    D = len(dims)
    h = 1.0 / dims[1]
    p = synth.base_params(D, list(dims), [O.AX_PERIODIC] * D, h)
    mu, rho = 3.0, 1.2
    p.update(mu_out=mu)
    H = O.Hierarchy(p, np.full(sum(O.face_counts(p)), rho), np.full(O.cell_count(p), mu),
                    np.full(sum(O.edge_counts(p)), mu))
    rng = np.random.default_rng(5)
    shape = tuple(reversed(dims))
    bs = [rng.standard_normal(shape) for _ in range(D)]
    x, st = H.solve(True, np.concatenate([b.ravel() for b in bs]), np.zeros(D * int(np.prod(dims))))
    assert st["status"] == 0
    # wavenumbers per axis (array axis order is z, y, x)
    ks = [2 * np.pi * np.fft.fftfreq(n, d=h) for n in dims]
    grids = np.meshgrid(*[ks[d] for d in reversed(range(D))], indexing="ij")
    kvec = [grids[D - 1 - d] for d in range(D)]
    s = [2 * np.sin(kd * h / 2) / h for kd in kvec]
    # lattice offsets: component a sits at vertex along a, centre along the others
    def phase(a):
        return np.exp(1j * sum(kvec[d] * (0.0 if d == a else 0.5 * h) for d in range(D)))
    bh = [np.fft.fftn(bs[a]) / phase(a) for a in range(D)]
    s2 = sum(sd * sd for sd in s)
    M = np.zeros(shape + (D, D))
    for a in range(D):
        for b in range(D):
            M[..., a, b] = p["inv_re"] * mu * s[a] * s[b]
        M[..., a, a] += p["sigma"] / p["dt"] * rho + p["inv_re"] * mu * s2
    uh = np.linalg.solve(M, np.stack(bh, axis=-1)[..., None])[..., 0]
    ue = [np.real(np.fft.ifftn(uh[..., a] * phase(a))) for a in range(D)]
    want = np.concatenate([u.ravel() for u in ue])
    assert np.linalg.norm(x - want) <= 1e-8 * np.linalg.norm(want)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("vel", [False, True])
def test_vcycles_reach_direct_solution(case, vel):
    c, H = hier(case)
    p = c["params"]
    A = H.csr(vel)
    n = A.shape[0]
    rng = np.random.default_rng(6)
    comp, pos = H.unknowns(vel)
    bvec = rng.standard_normal(n)
    singular = (not vel) and not any(p["axis_bc"][a] == O.AX_INOUT for a in range(p["dim"]))
    if singular:
        bvec -= bvec.mean()
    # compact layout in and out
    def to_compact(v):
        if vel:
            faces = [np.zeros(O.lattice_dims(p, O.FACE, a)[1][::-1]) for a in range(p["dim"])]
            for val, a, (i, j, k) in zip(v, comp, pos):
                faces[a][k, j, i] = val
            return np.concatenate([f.ravel() for f in faces])
        out = np.zeros(tuple(p["n"][:p["dim"]][::-1]) if p["dim"] == 3 else (p["n"][1], p["n"][0]))
        for val, (i, j, k) in zip(v, pos):
            out[(k, j, i) if p["dim"] == 3 else (j, i)] = val
        return out.ravel()
    bc = to_compact(bvec)
    xc, st = H.solve(vel, bc, np.zeros_like(bc))
    assert st["status"] == 0 and st["relres"] <= p["rtol"]
    Ad = A.toarray()
    if singular:
        Ad = Ad + np.ones((n, n)) * np.trace(Ad) / n ** 2
    xstar = np.linalg.solve(Ad, bvec)
    # map the compact result back to unknown order
    flat = to_compact(np.arange(n, dtype=float) + 1)
    lookup = {int(v) - 1: t for t, v in enumerate(flat) if v > 0}
    got = np.array([xc[lookup[r]] for r in range(n)])
    if singular:
        got -= got.mean()
        xstar -= xstar.mean()
    ev = np.abs(np.linalg.eigvals(Ad))
    cond = ev.max() / ev.min()
    err = np.linalg.norm(got - xstar) / np.linalg.norm(xstar)
    assert err <= cond * p["rtol"]


def test_constant_coefficient_convergence_factor():
    # textbook V(2,2) contraction for a Poisson problem is about 0.1
    p = synth.base_params(3, [16, 16, 32], [O.AX_WALLS, O.AX_WALLS, O.AX_INOUT], 1.0 / 16)
    H = O.Hierarchy(p, np.ones(sum(O.face_counts(p))), np.ones(O.cell_count(p)), np.ones(sum(O.edge_counts(p))))
    rng = np.random.default_rng(7)
    b = rng.standard_normal(O.cell_count(p))
    x, st = H.solve(False, b, np.zeros_like(b), hist_len=40)
    h = st["hist"]
    rate = (h[-1] / h[0]) ** (1.0 / (len(h) - 1))
    assert rate < 0.2, rate


def test_work_units_fall_with_levels():
    c = synth.channel_2d(seed=1)
    p = dict(c["params"])
    rho, mc, me = coefs_of(c)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(O.cell_count(p))
    b -= b.mean()
    wu = []
    for L in (1, 2, 3, 5):
        q = dict(p)
        q["max_levels"] = L
        q["max_cycles"] = 100000
        H = O.Hierarchy(q, rho, mc, me)
        x, st = H.solve(False, b, np.zeros_like(b))
        assert st["status"] == 0
        wu.append(st["work_units"])
    assert all(wu[i] > wu[i + 1] for i in range(len(wu) - 1)), wu
    assert wu[0] > 30 * wu[-1], wu
    assert wu[-1] < 300, wu


def test_condition_number_grows_like_h_minus_2():
    conds = []
    for n in (8, 16):
        p = synth.base_params(2, [2 * n, n], [O.AX_INOUT, O.AX_WALLS], 1.0 / n)
        H = O.Hierarchy(p, np.ones(sum(O.face_counts(p))), np.ones(O.cell_count(p)),
                        np.ones(sum(O.edge_counts(p))))
        ev = np.linalg.eigvalsh(H.csr(False).toarray())
        conds.append(ev[-1] / ev[0])
    assert 3.0 < conds[1] / conds[0] < 5.0, conds
