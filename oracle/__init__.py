"""FP64 CPU oracle for the immersed-boundary biofilm time step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product path never does.  It
shares no code with the HIP library in ``paper_1302_3663_amd``.

The numerical work lives in ``ibmg_oracle.c`` (plain loops, FP64, no fused
multiply-add); this module only marshals numpy arrays into it.  ``step.py``
strings the pieces together in the order of the paper's "Solution Strategy"
section.

Array conventions (the "compact" layout shared with the HIP library's
interface): a field on one lattice lists the closed-domain positions with x
fastest.  Along an axis a lattice is either cell-centred (n positions) or
vertex-centred (n + 1 positions, or n on a periodic axis).  Velocity-like
fields concatenate the D face lattices (faces normal to x, y, z); edge
fields concatenate the edge lattices parallel to x, y, z (2D: the single
corner lattice).
"""
import ctypes
import os

import numpy as np

from . import build as _build

AX_PERIODIC, AX_WALLS, AX_INOUT = 0, 1, 2
OK, EINVAL, ENOMEM, ENOCONV, ENUMERIC = 0, 1, 2, 3, 4


class Desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("axis_bc", ctypes.c_int * 3),
        ("h", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("inv_re", ctypes.c_double),
        ("force_coef", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("body_force", ctypes.c_double * 3),
        ("rho0", ctypes.c_double),
        ("rho_b", ctypes.c_double),
        ("d0_pow_d", ctypes.c_double),
        ("mu_out", ctypes.c_double),
        ("mu_max", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("kernel", ctypes.c_int),
        ("break_ratio", ctypes.c_double),
        ("nu1", ctypes.c_int),
        ("nu2", ctypes.c_int),
        ("max_levels", ctypes.c_int),
        ("max_cycles", ctypes.c_int),
        ("rtol", ctypes.c_double),
        ("gamma", ctypes.c_double * 16),
        ("decoupled", ctypes.c_int),
        ("galerkin", ctypes.c_int),
    ]


def make_desc(p):
    """Fill a Desc from a parameter dict (see paper_1302_3663_amd.synth)."""
    d = Desc()
    d.dim = p["dim"]
    for a in range(3):
        d.n[a] = p["n"][a] if a < p["dim"] else 1
        d.axis_bc[a] = p["axis_bc"][a] if a < p["dim"] else 0
        d.body_force[a] = p.get("body_force", [0.0, 0.0, 0.0])[a]
    for k in ("h", "sigma", "eps", "inv_re", "force_coef", "dt", "rho0", "rho_b", "d0_pow_d",
              "mu_out", "mu_max", "omega", "break_ratio", "rtol"):
        setattr(d, k, float(p[k]))
    for k in ("kernel", "nu1", "nu2", "max_levels", "max_cycles"):
        setattr(d, k, int(p[k]))
    g = p.get("gamma", [1.0] * 16)
    for l in range(16):
        d.gamma[l] = g[l] if l < len(g) else 1.0
    d.decoupled = int(p.get("decoupled", 0))
    d.galerkin = int(p.get("galerkin", 0))
    return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = ctypes.CDLL(path)
        D = ctypes.POINTER(Desc)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_long)
        u8 = ctypes.POINTER(ctypes.c_ubyte)
        vp = ctypes.c_void_p
        L.orc_phi.restype = ctypes.c_double
        L.orc_phi.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_phi_v.argtypes = [ctypes.c_int, dp, dp, ctypes.c_long]
        L.orc_lattice_count.restype = ctypes.c_long
        L.orc_lattice_count.argtypes = [D, ctypes.c_int, ctypes.c_int, ip]
        L.orc_spread_vec.argtypes = [D, ctypes.c_double, ctypes.c_long, dp, dp, dp]
        L.orc_interp_vec.argtypes = [D, ctypes.c_double, ctypes.c_long, dp, dp, dp]
        L.orc_density.argtypes = [D, ctypes.c_long, dp, dp]
        L.orc_viscosity.argtypes = [D, ctypes.c_int, ctypes.c_long, dp, dp]
        L.orc_springs.argtypes = [D, ctypes.c_long, dp, ctypes.c_long, ip, dp, dp, u8, dp, ctypes.c_int, lp]
        L.orc_fragments.argtypes = [ctypes.c_long, ctypes.c_long, ip, u8, u8, ip, lp, lp]
        L.orc_momentum_rhs.argtypes = [D, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        L.orc_momentum_apply_full.argtypes = [D, dp, dp, dp, dp, dp]
        L.orc_pressure_rhs.argtypes = [D, dp, dp]
        L.orc_divergence.argtypes = [D, dp, dp]
        L.orc_project.argtypes = [D, dp, dp, dp, dp]
        L.orc_hier_create.restype = vp
        L.orc_hier_create.argtypes = [D, dp, dp, dp, ip]
        L.orc_hier_destroy.argtypes = [vp]
        L.orc_hier_levels.argtypes = [vp, ip, lp]
        L.orc_solve.argtypes = [vp, ctypes.c_int, dp, dp, ip, dp, dp, dp, ctypes.c_int]
        L.orc_vcycles.argtypes = [vp, ctypes.c_int, dp, dp, ctypes.c_int]
        L.orc_solve_gcr.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ip, dp]
        L.orc_smooth.argtypes = [vp, ctypes.c_int, dp, dp, ctypes.c_int]
        L.orc_smooth_level.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int]
        L.orc_relres.restype = ctypes.c_double
        L.orc_relres.argtypes = [vp, ctypes.c_int, dp, dp]
        L.orc_csr_nnz.restype = ctypes.c_long
        L.orc_csr_nnz.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.orc_csr_export.restype = ctypes.c_long
        L.orc_csr_export.argtypes = [vp, ctypes.c_int, ctypes.c_int, lp, lp, dp]
        L.orc_unknowns.argtypes = [vp, ctypes.c_int, ctypes.c_int, ip, ip]
        L.orc_apply_vec.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_restrict_vec.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_prolong_vec.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_level_coefs.argtypes = [vp, ctypes.c_int, dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(st, what):
    if st != OK:
        raise RuntimeError(f"oracle {what} failed with status {st}")


# --------------------------------------------------------------------------
# lattice sizes
# --------------------------------------------------------------------------
CELL, FACE, EDGE = 0, 1, 2


def lattice_dims(p, kind, axis):
    d = make_desc(p)
    dims = (ctypes.c_int * 3)()
    n = lib().orc_lattice_count(ctypes.byref(d), kind, axis, dims)
    return n, tuple(dims)


def face_counts(p):
    return [lattice_dims(p, FACE, a)[0] for a in range(p["dim"])]


def edge_counts(p):
    axes = [0, 1, 2] if p["dim"] == 3 else [2]
    return [lattice_dims(p, EDGE, c)[0] for c in axes]


def cell_count(p):
    return lattice_dims(p, CELL, 0)[0]


def split_faces(p, v):
    out, off = [], 0
    for a, c in enumerate(face_counts(p)):
        _, dims = lattice_dims(p, FACE, a)
        out.append(v[off:off + c].reshape(dims[2], dims[1], dims[0]))
        off += c
    return out


# --------------------------------------------------------------------------
# regularised delta
# --------------------------------------------------------------------------
def phi(kernel, r):
    r = _f64(np.atleast_1d(r))
    out = np.empty_like(r)
    lib().orc_phi_v(kernel, _d(r), _d(out), r.size)
    return out


# --------------------------------------------------------------------------
# immersed boundary transfers
# --------------------------------------------------------------------------
def spread_vec(p, width, X, F):
    d = make_desc(p)
    X, F = _f64(X), _f64(F)
    eta = X.shape[1] if X.ndim == 2 else 0
    out = np.zeros(sum(face_counts(p)))
    _check(lib().orc_spread_vec(ctypes.byref(d), width, eta, _d(X), _d(F), _d(out)), "spread")
    return out


def interp_vec(p, width, X, u):
    d = make_desc(p)
    X, u = _f64(X), _f64(u)
    eta = X.shape[1]
    U = np.zeros((p["dim"], eta))
    _check(lib().orc_interp_vec(ctypes.byref(d), width, eta, _d(X), _d(u), _d(U)), "interp")
    return U


def density(p, X):
    d = make_desc(p)
    X = _f64(X)
    out = np.zeros(sum(face_counts(p)))
    _check(lib().orc_density(ctypes.byref(d), X.shape[1], _d(X), _d(out)), "density")
    return out


def viscosity_cells(p, X):
    d = make_desc(p)
    X = _f64(X)
    out = np.zeros(cell_count(p))
    _check(lib().orc_viscosity(ctypes.byref(d), 1, X.shape[1], _d(X), _d(out)), "viscosity")
    return out


def viscosity_edges(p, X):
    d = make_desc(p)
    X = _f64(X)
    out = np.zeros(sum(edge_counts(p)))
    _check(lib().orc_viscosity(ctypes.byref(d), 2, X.shape[1], _d(X), _d(out)), "viscosity")
    return out


def springs(p, X, ij, rest, K, alive, do_break=True):
    """Returns (F, alive_after, n_broken); alive is not modified in place."""
    d = make_desc(p)
    X = _f64(X)
    eta = X.shape[1]
    ij = np.ascontiguousarray(ij, dtype=np.int32)
    m = ij.shape[1]
    rest, K = _f64(rest), _f64(K)
    al = np.ascontiguousarray(alive, dtype=np.uint8).copy()
    F = np.zeros((p["dim"], eta))
    nb = ctypes.c_long(0)
    _check(lib().orc_springs(ctypes.byref(d), eta, _d(X), m, ij.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                             _d(rest), _d(K), al.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), _d(F),
                             1 if do_break else 0, ctypes.byref(nb)), "springs")
    return F, al, nb.value


def anchored_nodes(p, X0):
    """Nodes within the attachment distance of the attachment wall at t = 0
    (the low wall of axis attach_axis)."""
    ax = int(p.get("attach_axis", 1))
    return (np.asarray(X0, float)[ax] < float(p.get("attach_dist", 0.0))).astype(np.uint8)


def fragments(ij, alive, anchored):
    """Connected components of the alive springs: (label per node = smallest
    node id of its fragment, number of fragments, number of detached ones)."""
    ij = np.ascontiguousarray(ij, dtype=np.int32)
    m = ij.shape[1]
    anchored = np.ascontiguousarray(anchored, dtype=np.uint8)
    eta = anchored.size
    al = np.ascontiguousarray(alive, dtype=np.uint8)
    label = np.zeros(eta, np.int32)
    nf, nd = ctypes.c_long(0), ctypes.c_long(0)
    u8p = ctypes.POINTER(ctypes.c_ubyte)
    _check(lib().orc_fragments(eta, m, ij.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), al.ctypes.data_as(u8p),
                               anchored.ctypes.data_as(u8p), label.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                               ctypes.byref(nf), ctypes.byref(nd)), "fragments")
    return label, nf.value, nd.value


# --------------------------------------------------------------------------
# projection-step pieces
# --------------------------------------------------------------------------
def momentum_rhs(p, u, rho, mu_c, mu_e, f, with_boundary=True):
    d = make_desc(p)
    b = np.zeros(sum(face_counts(p)))
    _check(lib().orc_momentum_rhs(ctypes.byref(d), _d(_f64(u)), _d(_f64(rho)), _d(_f64(mu_c)), _d(_f64(mu_e)),
                                  _d(_f64(f)), _d(b), 1 if with_boundary else 0), "momentum_rhs")
    return b


def momentum_apply_full(p, u, rho, mu_c, mu_e):
    d = make_desc(p)
    y = np.zeros(sum(face_counts(p)))
    _check(lib().orc_momentum_apply_full(ctypes.byref(d), _d(_f64(u)), _d(_f64(rho)), _d(_f64(mu_c)),
                                         _d(_f64(mu_e)), _d(y)), "momentum_apply_full")
    return y


def pressure_rhs(p, ut):
    d = make_desc(p)
    b = np.zeros(cell_count(p))
    _check(lib().orc_pressure_rhs(ctypes.byref(d), _d(_f64(ut)), _d(b)), "pressure_rhs")
    return b


def divergence(p, u):
    d = make_desc(p)
    out = np.zeros(cell_count(p))
    _check(lib().orc_divergence(ctypes.byref(d), _d(_f64(u)), _d(out)), "divergence")
    return out


def project(p, ut, pres, rho):
    d = make_desc(p)
    u = np.zeros(sum(face_counts(p)))
    _check(lib().orc_project(ctypes.byref(d), _d(_f64(ut)), _d(_f64(pres)), _d(_f64(rho)), _d(u)), "project")
    return u


# --------------------------------------------------------------------------
# multigrid hierarchy
# --------------------------------------------------------------------------
class Hierarchy:
    """Coefficient hierarchy with assembled operators on every level."""

    def __init__(self, p, rho, mu_c, mu_e):
        self.p = p
        self._desc = make_desc(p)
        st = ctypes.c_int(0)
        self._rho, self._mc, self._me = _f64(rho), _f64(mu_c), _f64(mu_e)
        self.h = lib().orc_hier_create(ctypes.byref(self._desc), _d(self._rho), _d(self._mc), _d(self._me),
                                       ctypes.byref(st))
        _check(st.value, "hierarchy")
        dims = (ctypes.c_int * 48)()
        nunk = (ctypes.c_long * 32)()
        self.levels = lib().orc_hier_levels(self.h, dims, nunk)
        self.dims = [tuple(dims[3 * l:3 * l + 3]) for l in range(self.levels)]
        self.nunk = [(nunk[2 * l], nunk[2 * l + 1]) for l in range(self.levels)]

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_hier_destroy(self.h)
            self.h = None

    def solve(self, velocity, b, x0, hist_len=0):
        b = _f64(b)
        x = _f64(x0).copy()
        cyc = ctypes.c_int(0)
        rel = ctypes.c_double(0)
        wu = ctypes.c_double(0)
        hist = np.zeros(max(hist_len, 1))
        st = lib().orc_solve(self.h, int(velocity), _d(b), _d(x), ctypes.byref(cyc), ctypes.byref(rel),
                             ctypes.byref(wu), _d(hist), hist_len)
        return x, dict(status=st, cycles=cyc.value, relres=rel.value, work_units=wu.value,
                       hist=hist[:min(hist_len, cyc.value + 1)])

    def solve_gcr(self, velocity, b, x0, m=8, kmax=0):
        """V-cycle-preconditioned GCR(m); kmax > 0: exactly kmax iterations."""
        x = _f64(x0).copy()
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0)
        st = lib().orc_solve_gcr(self.h, int(velocity), int(m), int(kmax), _d(_f64(b)), _d(x), ctypes.byref(it),
                                 ctypes.byref(rel))
        return x, dict(status=st, cycles=it.value, relres=rel.value)

    def vcycles(self, velocity, b, x0, k):
        x = _f64(x0).copy()
        _check(lib().orc_vcycles(self.h, int(velocity), _d(_f64(b)), _d(x), k), "vcycles")
        return x

    def smooth(self, velocity, b, x0, k):
        x = _f64(x0).copy()
        _check(lib().orc_smooth(self.h, int(velocity), _d(_f64(b)), _d(x), k), "smooth")
        return x

    def smooth_level(self, velocity, level, b, x0, k):
        """k sweeps of the smoother of `level` on vectors of its unknowns."""
        x = _f64(x0).copy()
        _check(lib().orc_smooth_level(self.h, int(velocity), level, _d(_f64(b)), _d(x), k), "smooth_level")
        return x

    def relres(self, velocity, b, x):
        return lib().orc_relres(self.h, int(velocity), _d(_f64(b)), _d(_f64(x)))

    def csr(self, velocity, level=0):
        import scipy.sparse as sp
        nnz = lib().orc_csr_nnz(self.h, int(velocity), level)
        n = self.nunk[level][1 if velocity else 0]
        rp = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(max(nnz, 1), dtype=np.int64)
        val = np.zeros(max(nnz, 1))
        lp = ctypes.POINTER(ctypes.c_long)
        lib().orc_csr_export(self.h, int(velocity), level, rp.ctypes.data_as(lp), col.ctypes.data_as(lp), _d(val))
        return sp.csr_matrix((val[:nnz], col[:nnz], rp), shape=(n, n))

    def unknowns(self, velocity, level=0):
        n = self.nunk[level][1 if velocity else 0]
        comp = np.zeros(n, dtype=np.int32)
        pos = np.zeros((n, 3), dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        lib().orc_unknowns(self.h, int(velocity), level, comp.ctypes.data_as(ip), pos.ctypes.data_as(ip))
        return comp, pos

    def apply_vec(self, velocity, x, level=0):
        x = _f64(x)
        y = np.zeros_like(x)
        lib().orc_apply_vec(self.h, int(velocity), level, _d(x), _d(y))
        return y

    def restrict_vec(self, velocity, level, r):
        nc = self.nunk[level + 1][1 if velocity else 0]
        out = np.zeros(nc)
        lib().orc_restrict_vec(self.h, int(velocity), level, _d(_f64(r)), _d(out))
        return out

    def prolong_vec(self, velocity, level, xc):
        nf = self.nunk[level][1 if velocity else 0]
        out = np.zeros(nf)
        lib().orc_prolong_vec(self.h, int(velocity), level, _d(_f64(xc)), _d(out))
        return out

    def level_coefs(self, level):
        dims = self.dims[level]
        q = dict(self.p)
        q["n"] = list(dims)
        q["h"] = self.p["h"] * (2 ** level)
        rho = np.zeros(sum(face_counts(q)))
        mc = np.zeros(cell_count(q))
        me = np.zeros(sum(edge_counts(q)))
        lib().orc_level_coefs(self.h, level, _d(rho), _d(mc), _d(me))
        return rho, mc, me
