"""A solver context on one GPU: torch supplies the device memory (one
workspace tensor plus the caller's arrays) and the stream; every step runs in
libibmg.so through the C interface of include/ibmg.h.
"""
import ctypes

import torch

from . import _lib as L


def _chk(lib, st, where, ctx=None):
    if st != L.IBB_OK:
        msg = lib.ibb_status_string(st).decode()
        extra = lib.ibb_last_error(ctx)
        if extra:
            msg += ": " + extra.decode()
        raise L.IbbError(st, where, msg)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ctypes.c_void_p(t.data_ptr())


def lattice_count(params, kind, axis):
    lib = L.load()
    d = L.make_desc(params)
    n = ctypes.c_int64()
    dims = (ctypes.c_int * 3)()
    _chk(lib, lib.ibb_lattice_count(ctypes.byref(d), kind, axis, ctypes.byref(n), dims), "ibb_lattice_count")
    return n.value, tuple(dims)


def face_counts(params):
    return [lattice_count(params, 1, a)[0] for a in range(params["dim"])]


def edge_counts(params):
    return [lattice_count(params, 2, c)[0] for c in ([0, 1, 2] if params["dim"] == 3 else [2])]


def cell_count(params):
    return lattice_count(params, 0, 0)[0]


def footprint_bytes(params, max_nodes, max_springs, precision=L.IBB_FP64, inner_cycles=1):
    lib = L.load()
    d = L.make_desc(params, precision, inner_cycles)
    n = ctypes.c_size_t()
    _chk(lib, lib.ibb_footprint_bytes(ctypes.byref(d), max_nodes, max_springs, ctypes.byref(n)), "ibb_footprint_bytes")
    return n.value


def spread_static(params, width, X, F, out=None, stream=None, check=True):
    """ibb_spread_static: the spread of node vectors F [dim][n] at X to the
    face lattices (compact) without a context; the library's static scratch
    holds the bins.  Returns (out, status)."""
    lib = L.load()
    d = L.make_desc(params)
    dev = X.device
    if out is None:
        out = torch.zeros(sum(face_counts(params)), dtype=torch.float64, device=dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    st = lib.ibb_spread_static(ctypes.byref(d), float(width), X.shape[1], _ptr(X), _ptr(F), _ptr(out),
                               ctypes.c_void_p(s.cuda_stream))
    if check:
        _chk(lib, st, "ibb_spread_static")
    return out, st


class Context:
    """One biofilm problem resident on a GPU."""

    def __init__(self, params, max_nodes, max_springs, precision=L.IBB_FP64, inner_cycles=1, device="cuda:0",
                 stream=None):
        self.lib = L.load()
        self.params = dict(params)
        self.device = torch.device(device)
        self.desc = L.make_desc(params, precision, inner_cycles)
        self.precision, self.inner_cycles = precision, inner_cycles
        self.capacity = (int(max_nodes), int(max_springs))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = footprint_bytes(params, max_nodes, max_springs, precision, inner_cycles)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = ctypes.c_void_p()
        st = self.lib.ibb_create(ctypes.byref(self.desc), max_nodes, max_springs,
                                 ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.ctx))
        _chk(self.lib, st, "ibb_create")
        self.dim = params["dim"]
        self.n_face = sum(face_counts(params))
        self.n_cell = cell_count(params)
        self.n_edge = sum(edge_counts(params))
        self.eta = 0
        self.m = 0

    def close(self):
        if self.ctx:
            self.lib.ibb_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, n, dtype=torch.float64):
        return torch.zeros(n, dtype=dtype, device=self.device)

    def _c(self, st, where):
        _chk(self.lib, st, where, self.ctx)

    # ---- state ----
    def set_params(self, params):
        """Another problem of the same shape (see ibb_set_params)."""
        desc = L.make_desc(params, self.precision, self.inner_cycles)
        self._c(self.lib.ibb_set_params(self.ctx, ctypes.byref(desc)), "ibb_set_params")
        self.desc, self.params = desc, dict(params)

    def load(self, case):
        """Load a synthetic case (dict from synth) into this context and build
        its coefficients; the case must fit the context's shape and
        capacities."""
        dev = self.device
        self.set_params(case["params"])
        self.set_state(torch.as_tensor(case["u0"], dtype=torch.float64, device=dev).contiguous(),
                       torch.as_tensor(case["p0"], dtype=torch.float64, device=dev).contiguous())
        self.set_nodes(torch.as_tensor(case["X"], dtype=torch.float64, device=dev).contiguous())
        self.set_springs(torch.as_tensor(case["ij"], dtype=torch.int32, device=dev).contiguous(),
                         torch.as_tensor(case["rest"], dtype=torch.float64, device=dev).contiguous(),
                         torch.as_tensor(case["K"], dtype=torch.float64, device=dev).contiguous())
        self.update_coefficients()

    def set_state(self, u, p=None):
        self._c(self.lib.ibb_set_state(self.ctx, _ptr(u), _ptr(p)), "ibb_set_state")

    def get_state(self):
        u, p = self._new(self.n_face), self._new(self.n_cell)
        self._c(self.lib.ibb_get_state(self.ctx, _ptr(u), _ptr(p)), "ibb_get_state")
        return u, p

    def set_nodes(self, X):
        self.eta = X.shape[1]
        self._c(self.lib.ibb_set_nodes(self.ctx, self.eta, _ptr(X)), "ibb_set_nodes")

    def get_nodes(self):
        X = self._new(self.dim * self.eta).view(self.dim, self.eta)
        F = self._new(self.dim * self.eta).view(self.dim, self.eta)
        alive = self._new(max(self.m, 1), torch.uint8)[:self.m]
        self._c(self.lib.ibb_get_nodes(self.ctx, _ptr(X), _ptr(F), _ptr(alive) if self.m else None), "ibb_get_nodes")
        return X, F, alive

    def set_springs(self, ij, rest, K, alive=None):
        self.m = ij.shape[1]
        self._c(self.lib.ibb_set_springs(self.ctx, self.m, _ptr(ij), _ptr(rest), _ptr(K), _ptr(alive)),
                "ibb_set_springs")

    # ---- the step ----
    def update_coefficients(self):
        self._c(self.lib.ibb_update_coefficients(self.ctx), "ibb_update_coefficients")

    def projection_step(self, check=True):
        s = L.SolveStats()
        st = self.lib.ibb_projection_step(self.ctx, ctypes.byref(s))
        if check:
            self._c(st, "ibb_projection_step")
        out = {k: getattr(s, k) for k, _ in L.SolveStats._fields_}
        out["status"] = st
        return out

    def lagrangian_update(self):
        s = L.LagStats()
        self._c(self.lib.ibb_lagrangian_update(self.ctx, ctypes.byref(s)), "ibb_lagrangian_update")
        return {k: getattr(s, k) for k, _ in L.LagStats._fields_}

    # ---- individual steps ----
    def get_fields(self, level=0, levels_params=None):
        q = levels_params or self.params
        nf, nc, ne = sum(face_counts(q)), cell_count(q), sum(edge_counts(q))
        f = self._new(nf) if level == 0 else None
        rho, mc, me = self._new(nf), self._new(nc), self._new(ne)
        self._c(self.lib.ibb_get_fields(self.ctx, level, _ptr(f), _ptr(rho), _ptr(mc), _ptr(me)), "ibb_get_fields")
        return f, rho, mc, me

    def momentum_rhs(self):
        b = self._new(self.n_face)
        self._c(self.lib.ibb_momentum_rhs(self.ctx, _ptr(b)), "ibb_momentum_rhs")
        return b

    def pressure_rhs(self, ut):
        bp = self._new(self.n_cell)
        self._c(self.lib.ibb_pressure_rhs(self.ctx, _ptr(ut), _ptr(bp)), "ibb_pressure_rhs")
        return bp

    def mg_solve(self, which, b, x0, max_cycles=0, exact=0, check=True):
        x = x0.clone()
        cyc = ctypes.c_int()
        rel = ctypes.c_double()
        st = self.lib.ibb_mg_solve(self.ctx, which, _ptr(b), _ptr(x), max_cycles, exact, ctypes.byref(cyc),
                                   ctypes.byref(rel))
        if check:
            self._c(st, "ibb_mg_solve")
        return x, dict(status=st, cycles=cyc.value, relres=rel.value)

    def project(self, ut, p):
        u = self._new(self.n_face)
        self._c(self.lib.ibb_project(self.ctx, _ptr(ut), _ptr(p), _ptr(u)), "ibb_project")
        return u

    def interp(self, width, X, u):
        U = self._new(X.numel()).view(X.shape)
        self._c(self.lib.ibb_interp(self.ctx, width, X.shape[1], _ptr(X), _ptr(u), _ptr(U)), "ibb_interp")
        return U

    def spread(self, width, X, F):
        out = self._new(self.n_face)
        self._c(self.lib.ibb_spread(self.ctx, width, X.shape[1], _ptr(X), _ptr(F), _ptr(out)), "ibb_spread")
        return out

    def profile_enable(self, enable=True):
        self._c(self.lib.ibb_profile_enable(self.ctx, 1 if enable else 0), "ibb_profile_enable")

    def profile_read(self, kernel_class):
        n, ms, u = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_longlong()
        self._c(self.lib.ibb_profile_read(self.ctx, kernel_class, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(u)),
                "ibb_profile_read")
        return dict(launches=n.value, total_ms=ms.value, units=u.value)

    def level_info(self, level=0):
        nl = ctypes.c_int()
        n = (ctypes.c_int * 3)()
        self._c(self.lib.ibb_level_info(self.ctx, level, ctypes.byref(nl), n), "ibb_level_info")
        return nl.value, tuple(n)


def group_footprint_bytes(contexts):
    """ibb_group_footprint_bytes: the workspace a group of these contexts needs."""
    lib = L.load()
    n = len(contexts)
    arr = (L.CTX * n)(*[c.ctx.value for c in contexts])
    nbytes = ctypes.c_size_t()
    _chk(lib, lib.ibb_group_footprint_bytes(arr, n, ctypes.byref(nbytes)), "ibb_group_footprint_bytes")
    return nbytes.value


class Group:
    """Several contexts stepped together: their multigrid passes share
    launches and each solve tick is a replayed HIP graph.  The members must
    stay open while the group lives."""

    def __init__(self, contexts):
        self.lib = L.load()
        self.members = list(contexts)
        n = len(self.members)
        self._ctxs = (L.CTX * n)(*[c.ctx.value for c in self.members])
        nbytes = ctypes.c_size_t()
        st = self.lib.ibb_group_footprint_bytes(self._ctxs, n, ctypes.byref(nbytes))
        _chk(self.lib, st, "ibb_group_footprint_bytes")
        self.nbytes = nbytes.value
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.members[0].device)
        self.group = ctypes.c_void_p()
        st = self.lib.ibb_group_create(self._ctxs, n, ctypes.c_void_p(self.workspace.data_ptr()), self.nbytes,
                                       ctypes.byref(self.group))
        _chk(self.lib, st, "ibb_group_create")

    def _err(self, st, where):
        if st != L.IBB_OK:
            msg = self.lib.ibb_status_string(st).decode()
            extra = self.lib.ibb_group_last_error(self.group) if self.group else None
            if extra:
                msg += ": " + extra.decode()
            raise L.IbbError(st, where, msg)

    def projection_step(self, check=True):
        """check=True raises on any failure; check=False raises only on
        failures other than a member's non-convergence or non-finite
        residual, which its statistics record."""
        n = len(self.members)
        stats = (L.SolveStats * n)()
        st = self.lib.ibb_group_projection_step(self.group, stats)
        if check or st not in (L.IBB_OK, L.IBB_ENOCONV, L.IBB_ENUMERIC):
            self._err(st, "ibb_group_projection_step")
        out = []
        for s in stats:
            d = {k: getattr(s, k) for k, _ in L.SolveStats._fields_}
            out.append(d)
        return out

    def set_active(self, member, active):
        """Take member `member` out of the group's calls (False) or back in."""
        self._err(self.lib.ibb_group_set_active(self.group, int(member), 1 if active else 0), "ibb_group_set_active")

    def lagrangian_update(self):
        n = len(self.members)
        stats = (L.LagStats * n)()
        self._err(self.lib.ibb_group_lagrangian_update(self.group, stats), "ibb_group_lagrangian_update")
        return [{k: getattr(s, k) for k, _ in L.LagStats._fields_} for s in stats]

    def close(self):
        if self.group:
            self.lib.ibb_group_destroy(self.group)
            self.group = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_case(case, precision=L.IBB_FP64, inner_cycles=1, device="cuda:0", spare_nodes=0):
    """Context loaded with a synthetic case (dict from synth) and coefficients built."""
    p = case["params"]
    X = torch.as_tensor(case["X"], dtype=torch.float64, device=device).contiguous()
    ij = torch.as_tensor(case["ij"], dtype=torch.int32, device=device).contiguous()
    ctx = Context(p, X.shape[1] + spare_nodes, max(ij.shape[1], 1), precision, inner_cycles, device)
    ctx.set_state(torch.as_tensor(case["u0"], dtype=torch.float64, device=device).contiguous(),
                  torch.as_tensor(case["p0"], dtype=torch.float64, device=device).contiguous())
    ctx.set_nodes(X)
    ctx.set_springs(ij, torch.as_tensor(case["rest"], dtype=torch.float64, device=device).contiguous(),
                    torch.as_tensor(case["K"], dtype=torch.float64, device=device).contiguous())
    ctx.update_coefficients()
    return ctx
