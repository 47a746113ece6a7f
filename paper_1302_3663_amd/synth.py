"""Seeded synthetic inputs shaped like the paper's biofilm workloads.

This module only draws inputs: node positions, spring lists, stiffnesses,
initial and boundary velocities, and the parameter set of each workload.  It
holds none of the method's arithmetic (no delta kernels, stencils or solves)
and is the one module that both the HIP path and the CPU oracle read.

Nondimensional constants follow the paper's scaling table (L = 50 um,
u0 = 1e-3 m/s, T = 1 s, rho0 = 998 kg/m^3, mu = 1e-3 kg/(m s),
pressure drop 0.8144 Pa): sigma = L / (T u0) = 0.05,
eps = dp / (rho0 u0^2) = 816.03, Re = rho0 L u0 / mu = 0.0499.
The paper's microscopy cell coordinates are not available, so node clouds are
drawn from the shapes and spacings it describes (mounds and films on the
bottom wall, about 1 um between cells, springs to neighbours within a few um).
"""
import functools
import math

import numpy as np

AX_PERIODIC, AX_WALLS, AX_INOUT = 0, 1, 2

L_CHAR = 50e-6
SIGMA = L_CHAR / (1.0 * 1e-3)
EPS = 0.8144 / (998.0 * 1e-6)
RE = 998.0 * L_CHAR * 1e-3 / 1e-3


def base_params(dim, n, axis_bc, h):
    return dict(
        dim=dim, n=list(n) + [1] * (3 - len(n)), axis_bc=list(axis_bc) + [0] * (3 - len(axis_bc)), h=h,
        sigma=SIGMA, eps=EPS, inv_re=1.0 / RE, force_coef=1.0, dt=1e-4,
        body_force=[0.0, 0.0, 0.0], rho0=1.0, rho_b=0.0, d0_pow_d=0.0,
        mu_out=1.0, mu_max=1.0, omega=0.02, kernel=0, break_ratio=2.0,
        nu1=2, nu2=2, max_levels=0, max_cycles=200, rtol=1e-10, gamma=[1.0] * 16,
        track_fragments=0, attach_axis=1, attach_dist=0.0, decoupled=0,
    )


# --------------------------------------------------------------------------
# node clouds
# --------------------------------------------------------------------------
def half_disc_uniform(rng, n, cx, r):
    """n points uniform in the half-disc of radius r centred at (cx, 0), y >= 0."""
    xs, ys, have = [], [], 0
    while have < n:
        x = rng.uniform(-r, r, size=4 * n)
        y = rng.uniform(0.0, r, size=4 * n)
        ok = x * x + y * y < r * r
        take = min(n - have, int(ok.sum()))
        xs.append(cx + x[ok][:take])
        ys.append(y[ok][:take])
        have += take
    return np.array([np.concatenate(xs), np.concatenate(ys)])


def poisson_disc(rng, inside, lo, hi, rmin, limit, seed_point, k=30):
    """Bridson's dart throwing grown from seed_point: points at least rmin
    apart inside the region given by the vectorised predicate inside(P),
    within the box [lo, hi]; growth stops at `limit` points."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    D = lo.size
    cs = rmin / math.sqrt(D)
    shape = np.maximum(1, np.ceil((hi - lo) / cs).astype(int))
    grid = -np.ones(tuple(shape), dtype=np.int64)
    P = np.empty((max(int(limit), 1), D))
    P[0] = np.asarray(seed_point, float)
    n = 1
    grid[tuple(np.minimum(((P[0] - lo) / cs).astype(int), shape - 1))] = 0
    active = [0]
    reach = int(math.ceil(math.sqrt(D))) + 1
    while active and n < limit:
        ai = rng.integers(len(active))
        base = P[active[ai]]
        # k candidates in the shell [rmin, 2 rmin)
        dirs = rng.normal(size=(k, D))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        rad = rmin * (1.0 + rng.random(k))
        cand = base + dirs * rad[:, None]
        ok_box = np.all((cand >= lo) & (cand <= hi), axis=1)
        ok_in = np.zeros(k, bool)
        if ok_box.any():
            ok_in[ok_box] = inside(cand[ok_box])
        placed = False
        for c in cand[ok_in]:
            gi = np.minimum(((c - lo) / cs).astype(int), shape - 1)
            sl = tuple(slice(max(0, g - reach), min(s, g + reach + 1)) for g, s in zip(gi, shape))
            near = grid[sl]
            near = near[near >= 0]
            if near.size:
                dd = np.linalg.norm(P[near] - c, axis=1)
                if np.any(dd < rmin):
                    continue
            grid[tuple(gi)] = n
            P[n] = c
            active.append(n)
            n += 1
            placed = True
            break
        if not placed:
            active.pop(ai)
    return P[:n].T.copy()


def poisson_disc_batched(rng, inside, lo, hi, rmin, limit, batch=400000, max_rounds=400):
    """Random sequential addition in batches (for large node counts): each
    round draws uniform candidates in the box, keeps those inside the region
    and at least rmin from every accepted point, drops the later one of every
    pair of candidates closer than rmin, and accepts the rest; stops at
    `limit` points or after max_rounds.  Points end up at least rmin apart."""
    from scipy.spatial import cKDTree
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    D = lo.size
    acc = np.empty((0, D))
    for _ in range(max_rounds):
        if len(acc) >= limit:
            break
        cand = lo + (hi - lo) * rng.random((batch, D))
        cand = cand[inside(cand)]
        if len(acc) and len(cand):
            d, _ = cKDTree(acc).query(cand, k=1, distance_upper_bound=rmin)
            cand = cand[~(d < rmin)]
        if len(cand) > 1:
            pairs = cKDTree(cand).query_pairs(rmin, output_type="ndarray")
            if len(pairs):
                keep = np.ones(len(cand), bool)
                keep[pairs.max(axis=1)] = False
                cand = cand[keep]
        acc = np.vstack([acc, cand[:limit - len(acc)]])
    return acc.T.copy()


def spring_pairs(X, cutoff):
    """All node pairs closer than cutoff (strictly), as int32 [2][m], i < j."""
    from scipy.spatial import cKDTree
    pairs = cKDTree(X.T).query_pairs(cutoff, output_type="ndarray")
    if pairs.size == 0:
        return np.zeros((2, 0), np.int32)
    d = np.linalg.norm(X[:, pairs[:, 0]] - X[:, pairs[:, 1]], axis=0)
    pairs = pairs[d < cutoff]
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    return np.ascontiguousarray(pairs[order].T.astype(np.int32))


def rest_lengths(X, ij):
    return np.linalg.norm(X[:, ij[1]] - X[:, ij[0]], axis=0)


# --------------------------------------------------------------------------
# boundary and initial velocity data
# --------------------------------------------------------------------------
def face_dims(p, a):
    """Closed-domain extent of the a-face lattice along x, y, z."""
    dims = []
    for d in range(3):
        if d >= p["dim"]:
            dims.append(1)
        elif d == a:
            dims.append(p["n"][d] if p["axis_bc"][d] == AX_PERIODIC else p["n"][d] + 1)
        else:
            dims.append(p["n"][d])
    return dims


def duct_profile(nx, ny, h, terms=199):
    """Laminar axial velocity in a square duct (Spiga-Morini double series),
    at cell centres of an nx x ny cross-section, scaled to 1 at the centre."""
    return _duct_profile(int(nx), int(ny), float(h), int(terms)).copy()


@functools.lru_cache(maxsize=16)
def _duct_profile(nx, ny, h, terms):
    ax, ay = nx * h, ny * h
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    s = np.zeros((ny, nx))
    s0 = 0.0
    for nn in range(1, terms + 1, 2):
        sx = np.sin(nn * math.pi * x / ax)
        for mm in range(1, terms + 1, 2):
            c = 1.0 / (nn * mm * (nn * nn + mm * mm))
            s += c * np.outer(np.sin(mm * math.pi * y / ay), sx)
            s0 += c * math.sin(nn * math.pi / 2) * math.sin(mm * math.pi / 2)
    return s / s0


def initial_velocity(p, umax=1.0):
    """Laminar flow in the channel (2D: parabola across y; 3D: duct profile
    along z), written on every face of the flow component including the
    inflow face; other components zero."""
    comps = []
    for a in range(p["dim"]):
        comps.append(np.zeros(face_dims(p, a)[::-1]))
    h = p["h"]
    if p["dim"] == 2:
        ly = p["n"][1] * h
        y = (np.arange(p["n"][1]) + 0.5) * h
        prof = umax * 4.0 * y * (ly - y) / (ly * ly)
        comps[0][:] = prof[None, :, None]
    else:
        prof = umax * duct_profile(p["n"][0], p["n"][1], h)
        comps[2][:, :, :] = prof[None, :, :]
    return np.concatenate([c.ravel() for c in comps])


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def _finish(p, X, ij, K, region_measure, rng):
    eta = X.shape[1]
    p["d0_pow_d"] = region_measure / max(eta, 1)
    rest = rest_lengths(X, ij) if ij.shape[1] else np.zeros(0)
    n_cells = int(np.prod(p["n"][:p["dim"]]))
    return dict(params=p, u0=initial_velocity(p), p0=np.zeros(n_cells), X=X, ij=ij, rest=rest,
                K=np.asarray(K, float), seed=None)


def channel_2d(seed=1, nx=64, ny=32, eta=200, radius=0.25, cutoff=0.08):
    """2D channel, periodic in x with walls in y, driven by a body force that
    makes the unit-peak parabola the biofilm-free steady state; uniform nodes
    in a half-disc on the bottom wall."""
    rng = np.random.default_rng(seed)
    h = 1.0 / ny
    p = base_params(2, [nx, ny], [AX_PERIODIC, AX_WALLS], h)
    ly = ny * h
    p["body_force"] = [8.0 * 1.0 * p["mu_out"] * p["inv_re"] / (ly * ly), 0.0, 0.0]
    p.update(rho_b=0.1, mu_max=10.0, omega=0.02, break_ratio=1.5)
    X = half_disc_uniform(rng, eta, 0.5 * nx * h, radius)
    p["attach_dist"] = math.sqrt(0.5 * math.pi * radius * radius / eta)
    ij = spring_pairs(X, cutoff)
    K = np.full(ij.shape[1], 1e2)
    out = _finish(p, X, ij, K, 0.5 * math.pi * radius * radius, rng)
    out["seed"] = seed
    return out


def _mound_inside(H, s, cx, cz):
    def inside(P):
        x, y, z = P[:, 0], P[:, 1], P[:, 2]
        return (y >= 0.0) & (y <= H * np.exp(-((x - cx) ** 2 + (z - cz) ** 2) / (2 * s * s)))
    return inside


def _mound_volume(H, s):
    return H * 2.0 * math.pi * s * s


def _union_volume(H, s, centres, Lz, nx=1024):
    """Volume under the highest of several Gaussian mounds on [0,1] x [0,Lz]
    (midpoint rule)."""
    x = (np.arange(nx) + 0.5) / nx
    nz = int(nx * Lz)
    z = (np.arange(nz) + 0.5) * (Lz / nz)
    top = np.zeros((nz, nx))
    for cz in centres:
        top = np.maximum(top, H * np.exp(-((x[None, :] - 0.5) ** 2 + (z[:, None] - cz) ** 2) / (2 * s * s)))
    return float(top.sum() * (1.0 / nx) * (Lz / nz))


def tube_3d(seed=2, n=(64, 64, 128), eta=5000, spacing=0.02, cutoff=0.05, rho_b=0.05, mu_max=100.0,
            omega=0.01, mounds=1, K_range=None, H=0.3, s=0.18, nu=(2, 2), gamma_2h=1.0):
    """3D square tube: walls in x and y, laminar inflow at z = 0 and a free
    outflow at z = Lz; Poisson-disc nodes filling Gaussian mounds on the
    bottom wall y = 0.  gamma_2h scales the viscosity restricted to the first
    coarse level (eq:ViscCoarseGrid); coarser levels inherit it through the
    restriction."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n[0]
    p = base_params(3, list(n), [AX_WALLS, AX_WALLS, AX_INOUT], h)
    p.update(rho_b=rho_b, mu_max=mu_max, omega=omega, break_ratio=2.0, nu1=nu[0], nu2=nu[1], attach_dist=spacing)
    p["gamma"] = [1.0, gamma_2h] + [1.0] * 14
    Lz = n[2] * h
    if mounds == 1:
        cz = 0.5 * Lz
        inside = _mound_inside(H, s, 0.5, cz)
        lo = [max(0.0, 0.5 - 3 * s), 0.0, max(0.0, cz - 3 * s)]
        hi = [min(1.0, 0.5 + 3 * s), H, min(Lz, cz + 3 * s)]
        X = poisson_disc(rng, inside, lo, hi, spacing, eta, [0.5, 0.25 * spacing, cz])
    else:
        # overlapping mounds: one process over their union keeps the minimum
        # spacing everywhere; it grows from the base of the middle mound
        parts = [_mound_inside(H, s, 0.5, Lz * (m + 1) / (mounds + 1)) for m in range(mounds)]

        def inside(P):
            ok = parts[0](P)
            for f in parts[1:]:
                ok |= f(P)
            return ok
        X = poisson_disc(rng, inside, [0.0, 0.0, 0.0], [1.0, H, Lz], spacing, eta,
                         [0.5, 0.25 * spacing, Lz * ((mounds + 1) // 2) / (mounds + 1)])
    ij = spring_pairs(X, cutoff)
    if K_range is None:
        K = np.full(ij.shape[1], 1e2)
    else:
        K = 10.0 ** rng.uniform(math.log10(K_range[0]), math.log10(K_range[1]), size=ij.shape[1])
    if mounds == 1:
        vol = _mound_volume(H, s)
    else:
        # the process stops at eta nodes: the biofilm is the part of the
        # union it filled, measured by the nodes' own packing density
        full = _union_volume(H, s, [Lz * (m + 1) / (mounds + 1) for m in range(mounds)], Lz)
        vol = full * min(1.0, X.shape[1] / eta)
    out = _finish(p, X, ij, K, vol, rng)
    out["seed"] = seed
    return out


def tiny_2d(seed=11, nx=16, ny=8, eta=12, inout=False):
    """Small 2D case for the oracle tests (a few tiles, a handful of nodes)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / ny
    bc = [AX_INOUT, AX_WALLS] if inout else [AX_PERIODIC, AX_WALLS]
    p = base_params(2, [nx, ny], bc, h)
    if not inout:
        p["body_force"] = [8.0 * p["mu_out"] * p["inv_re"], 0.0, 0.0]
    p.update(rho_b=0.1, mu_max=10.0, omega=0.12, break_ratio=1.5, attach_dist=0.1)
    X = half_disc_uniform(rng, eta, 0.5 * nx * h, 0.3)
    ij = spring_pairs(X, 0.2)
    K = np.full(ij.shape[1], 1e2)
    out = _finish(p, X, ij, K, 0.5 * math.pi * 0.09, rng)
    if inout:
        ly = ny * h
        y = (np.arange(ny) + 0.5) * h
        prof = 4.0 * y * (ly - y) / (ly * ly)
        u = np.zeros((ny, nx + 1))
        u[:, :] = prof[:, None]
        out["u0"] = np.concatenate([u.ravel(), np.zeros(nx * (ny + 1))])
    out["seed"] = seed
    return out


def tiny_3d(seed=12, n=(8, 8, 16), eta=20, periodic_z=False, periodic_x=False):
    """Small 3D tube for the oracle tests (walls in x and y, inflow and
    outflow in z; x and z periodic on request)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n[0]
    bc = [AX_PERIODIC if periodic_x else AX_WALLS, AX_WALLS, AX_PERIODIC if periodic_z else AX_INOUT]
    p = base_params(3, list(n), bc, h)
    if periodic_z:
        p["body_force"] = [0.0, 0.0, 1.0]
    p.update(rho_b=0.05, mu_max=20.0, omega=0.15, break_ratio=2.0, attach_dist=0.09)
    Lz = n[2] * h
    inside = _mound_inside(0.4, 0.2, 0.5, 0.5 * Lz)
    X = poisson_disc(rng, inside, [0.1, 0.0, 0.5 * Lz - 0.6], [0.9, 0.4, 0.5 * Lz + 0.6], 0.09, eta,
                     [0.5, 0.02, 0.5 * Lz])
    ij = spring_pairs(X, 0.2)
    K = np.full(ij.shape[1], 50.0)
    out = _finish(p, X, ij, K, _mound_volume(0.4, 0.2), rng)
    out["seed"] = seed
    return out


def rough_thickness(rng, modes, mean, amp, Lx, Lz):
    """Film thickness mean * (1 + amp * xi(x, z)) with xi a sum of `modes`
    random Fourier modes (integer wavenumbers up to 4 across the wall, random
    phases and weights), scaled so that max |xi| = 1 on a fine sample."""
    kx = rng.integers(0, 5, size=modes)
    kz = rng.integers(1, 9, size=modes)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    wt = rng.uniform(0.5, 1.0, size=modes)

    def raw(x, z):
        v = np.zeros(np.broadcast(x, z).shape)
        for a, b, c, w in zip(kx, kz, ph, wt):
            v += w * np.cos(2.0 * math.pi * (a * x / Lx + b * z / Lz) + c)
        return v
    xs = np.linspace(0.0, Lx, 257)
    zs = np.linspace(0.0, Lz, 513)
    scale = np.max(np.abs(raw(xs[None, :], zs[:, None])))

    def thickness(x, z):
        return mean * (1.0 + amp * raw(x, z) / scale)
    return thickness


def film_3d(seed=5, n=(256, 256, 512), eta=200000, spacing=0.008, rho_b=0.3, mu_max=1e3, omega=0.01,
            gamma_2h=0.7):
    """3D tube (walls in x and y, laminar inflow at z = 0, free outflow) with
    a rough biofilm film on the bottom wall y = 0: thickness 20 h (1 + xi / 2)
    with xi an 8-mode random Fourier field in [-1, 1], Poisson-disc nodes at
    the given spacing filling it, springs within 2.5 spacings, fragments
    tracked."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n[0]
    p = base_params(3, list(n), [AX_WALLS, AX_WALLS, AX_INOUT], h)
    p.update(rho_b=rho_b, mu_max=mu_max, omega=omega, break_ratio=2.0, attach_dist=spacing, track_fragments=1)
    p["gamma"] = [1.0, gamma_2h] + [1.0] * 14
    Lz = n[2] * h
    top = rough_thickness(rng, 8, 20.0 * h, 0.5, 1.0, Lz)

    def inside(P):
        return (P[:, 1] >= 0.0) & (P[:, 1] <= top(P[:, 0], P[:, 2]))
    X = poisson_disc_batched(rng, inside, [0.0, 0.0, 0.0], [1.0, 1.5 * 20.0 * h, Lz], spacing, eta)
    ij = spring_pairs(X, 2.5 * spacing)
    K = np.full(ij.shape[1], 1e2)
    xs = (np.arange(512) + 0.5) / 512
    zs = (np.arange(1024) + 0.5) * (Lz / 1024)
    film = float(np.mean(top(xs[None, :], zs[:, None])) * Lz)
    out = _finish(p, X, ij, K, film * min(1.0, X.shape[1] / eta), rng)
    out["seed"] = seed
    out["film_volume"] = film
    return out


# --------------------------------------------------------------------------
# serving stream
# --------------------------------------------------------------------------
SERVING_SIZES = [(32, 32), (64, 32), (128, 64), (32, 32, 32), (64, 64, 64), (64, 64, 128)]


def jittered_mound(rng, H, s, cx, cz, Lz, spacing, eta, jitter=0.15):
    """Up to eta points on a lattice of the given spacing, each moved by at
    most jitter*spacing per axis, kept inside the Gaussian mound (so any two
    points are at least (1 - 2 jitter) spacing apart); nearest the mound's
    axis first."""
    xs = np.arange(spacing / 2, 1.0, spacing)
    ys = np.arange(spacing / 2, H, spacing)
    zs = np.arange(spacing / 2, Lz, spacing)
    P = np.stack(np.meshgrid(xs, ys, zs, indexing="ij"), axis=-1).reshape(-1, 3)
    P = P + rng.uniform(-jitter * spacing, jitter * spacing, size=P.shape)
    ok = (P[:, 1] >= 0) & (P[:, 1] <= H * np.exp(-((P[:, 0] - cx) ** 2 + (P[:, 2] - cz) ** 2) / (2 * s * s)))
    P = P[ok & (P[:, 0] > 0) & (P[:, 0] < 1) & (P[:, 2] > 0) & (P[:, 2] < Lz)]
    r2 = (P[:, 0] - cx) ** 2 + (P[:, 2] - cz) ** 2 + P[:, 1] ** 2
    P = P[np.argsort(r2, kind="stable")][:eta]
    return P.T.copy()


def serving_request(j, steps=10):
    """Request j of the serving stream (seed 1000 + j): a grid drawn from
    SERVING_SIZES (2D as the channel, 3D as the tube), a log-uniform node
    count in [100, 10000], a log-uniform viscosity ratio in [1, 1e3] and a
    uniform density ratio in [1, 1.3].  Springs join nodes closer than 2.5
    mean spacings (2D) or 2 lattice spacings (3D)."""
    rng = np.random.default_rng(1000 + j)
    size = SERVING_SIZES[int(rng.integers(len(SERVING_SIZES)))]
    eta = int(round(10 ** rng.uniform(2.0, 4.0)))
    mu_max = float(10 ** rng.uniform(0.0, 3.0))
    rho_b = float(rng.uniform(1.0, 1.3)) - 1.0
    if len(size) == 2:
        nx, ny = size
        h = 1.0 / ny
        p = base_params(2, [nx, ny], [AX_PERIODIC, AX_WALLS], h)
        ly = ny * h
        p["body_force"] = [8.0 * p["mu_out"] * p["inv_re"] / (ly * ly), 0.0, 0.0]
        p.update(rho_b=rho_b, mu_max=mu_max, omega=0.02, break_ratio=1.5)
        radius = 0.25
        X = half_disc_uniform(rng, eta, 0.5 * nx * h, radius)
        area = 0.5 * math.pi * radius * radius
        p["attach_dist"] = math.sqrt(area / eta)
        ij = spring_pairs(X, 2.5 * math.sqrt(area / eta))
        out = _finish(p, X, ij, np.full(ij.shape[1], 1e2), area, rng)
    else:
        n = list(size)
        h = 1.0 / n[0]
        p = base_params(3, n, [AX_WALLS, AX_WALLS, AX_INOUT], h)
        p.update(rho_b=rho_b, mu_max=mu_max, omega=0.01, break_ratio=2.0)
        Lz = n[2] * h
        H, sw = 0.3, 0.18
        vol = _mound_volume(H, sw)
        spacing = 0.9 * (vol / eta) ** (1.0 / 3.0)
        X = jittered_mound(rng, H, sw, 0.5, 0.5 * Lz, Lz, spacing, eta)
        p["attach_dist"] = spacing
        ij = spring_pairs(X, 2.0 * spacing)
        out = _finish(p, X, ij, np.full(ij.shape[1], 1e2), vol * X.shape[1] / eta, rng)
    out["seed"] = 1000 + j
    out["steps"] = steps
    out["size"] = size
    return out


WORKLOADS = {
    "channel2d_64x32": lambda: channel_2d(seed=1),
    # the tubes scale the coarse viscosity by 0.7 (the lower end of the range
    # the paper reports as fastest); measured: about 30% fewer cycles than 1
    "tube3d_64x64x128": lambda: tube_3d(seed=2, gamma_2h=0.7),
    "tube3d_128x128x256": lambda: tube_3d(seed=3, n=(128, 128, 256), eta=50000, mounds=3, rho_b=0.2,
                                          mu_max=1e3, K_range=(1e1, 1e3), H=0.62, s=0.31, nu=(3, 3), gamma_2h=0.7),
    "film3d_256x256x512": lambda: film_3d(),
}
