"""ctypes binding of include/ibmg.h (argument marshalling only).

Every computation runs in libibmg.so.  If the library has not been built the
loader raises: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))

IBB_OK, IBB_EINVAL, IBB_ENOMEM, IBB_ENOCONV, IBB_ENUMERIC, IBB_EDEVICE, IBB_ESTATE = range(7)
IBB_AXIS_PERIODIC, IBB_AXIS_WALLS, IBB_AXIS_INOUT = 0, 1, 2
IBB_FP64, IBB_FP32_REFINED = 0, 1


class IbbError(RuntimeError):
    def __init__(self, status, where, msg=""):
        self.status = status
        super().__init__(f"{where}: status {status} ({msg})")


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
        ("precision", ctypes.c_int),
        ("inner_cycles", ctypes.c_int),
        ("wg_coarse_max", ctypes.c_int),
        ("track_fragments", ctypes.c_int),
        ("attach_axis", ctypes.c_int),
        ("attach_dist", ctypes.c_double),
        ("krylov_restart", ctypes.c_int),
        ("smoother_passes", ctypes.c_int),
        ("decoupled", ctypes.c_int),
        ("coarse_tail", ctypes.c_int),
        ("smoother_zblock", ctypes.c_int),
        ("galerkin", ctypes.c_int),
    ]


class SolveStats(ctypes.Structure):
    _fields_ = [
        ("status_u", ctypes.c_int), ("status_p", ctypes.c_int),
        ("cycles_u", ctypes.c_int), ("cycles_p", ctypes.c_int),
        ("vcycles_u", ctypes.c_int), ("vcycles_p", ctypes.c_int),
        ("relres_u", ctypes.c_double), ("relres_p", ctypes.c_double),
        ("t_u_ms", ctypes.c_double), ("t_p_ms", ctypes.c_double),
        ("dof_u", ctypes.c_longlong), ("dof_p", ctypes.c_longlong),
    ]


class LagStats(ctypes.Structure):
    _fields_ = [("n_broken", ctypes.c_int), ("n_alive", ctypes.c_int), ("t_ms", ctypes.c_double),
                ("n_fragments", ctypes.c_int), ("n_detached", ctypes.c_int)]


def make_desc(p, precision=IBB_FP64, inner_cycles=1):
    d = Desc()
    d.dim = p["dim"]
    for a in range(3):
        d.n[a] = p["n"][a] if a < p["dim"] else 1
        d.axis_bc[a] = p["axis_bc"][a] if a < p["dim"] else 0
        d.body_force[a] = p.get("body_force", [0.0] * 3)[a]
    for k in ("h", "sigma", "eps", "inv_re", "force_coef", "dt", "rho0", "rho_b", "d0_pow_d", "mu_out", "mu_max",
              "omega", "break_ratio", "rtol"):
        setattr(d, k, float(p[k]))
    for k in ("kernel", "nu1", "nu2", "max_levels", "max_cycles"):
        setattr(d, k, int(p[k]))
    g = p.get("gamma", [1.0] * 16)
    for l in range(16):
        d.gamma[l] = g[l] if l < len(g) else 1.0
    d.precision = int(p.get("precision", precision))
    d.inner_cycles = int(p.get("inner_cycles", inner_cycles))
    d.wg_coarse_max = int(p.get("wg_coarse_max", 0))
    d.track_fragments = int(p.get("track_fragments", 0))
    d.attach_axis = int(p.get("attach_axis", 1))
    d.attach_dist = float(p.get("attach_dist", 0.0))
    d.krylov_restart = int(p.get("krylov_restart", 0))
    d.smoother_passes = int(p.get("smoother_passes", 0))
    d.decoupled = int(p.get("decoupled", 0))
    d.coarse_tail = int(p.get("coarse_tail", 0))
    d.smoother_zblock = int(p.get("smoother_zblock", 0))
    d.galerkin = int(p.get("galerkin", 0))
    return d


VP = ctypes.c_void_p
I64 = ctypes.c_int64
DESC = ctypes.POINTER(Desc)
CTX = ctypes.c_void_p

# name -> (restype, argtypes); every function declared in include/ibmg.h
ABI_FUNCTIONS = {
    "ibb_lattice_count": (ctypes.c_int, [DESC, ctypes.c_int, ctypes.c_int, ctypes.POINTER(I64),
                                         ctypes.POINTER(ctypes.c_int)]),
    "ibb_footprint_bytes": (ctypes.c_int, [DESC, I64, I64, ctypes.POINTER(ctypes.c_size_t)]),
    "ibb_create": (ctypes.c_int, [DESC, I64, I64, VP, ctypes.c_size_t, VP, ctypes.POINTER(CTX)]),
    "ibb_destroy": (ctypes.c_int, [CTX]),
    "ibb_set_state": (ctypes.c_int, [CTX, VP, VP]),
    "ibb_set_params": (ctypes.c_int, [CTX, ctypes.POINTER(Desc)]),
    "ibb_get_state": (ctypes.c_int, [CTX, VP, VP]),
    "ibb_set_nodes": (ctypes.c_int, [CTX, I64, VP]),
    "ibb_get_nodes": (ctypes.c_int, [CTX, VP, VP, VP]),
    "ibb_set_springs": (ctypes.c_int, [CTX, I64, VP, VP, VP, VP]),
    "ibb_update_coefficients": (ctypes.c_int, [CTX]),
    "ibb_projection_step": (ctypes.c_int, [CTX, ctypes.POINTER(SolveStats)]),
    "ibb_lagrangian_update": (ctypes.c_int, [CTX, ctypes.POINTER(LagStats)]),
    "ibb_get_fields": (ctypes.c_int, [CTX, ctypes.c_int, VP, VP, VP, VP]),
    "ibb_momentum_rhs": (ctypes.c_int, [CTX, VP]),
    "ibb_pressure_rhs": (ctypes.c_int, [CTX, VP, VP]),
    "ibb_mg_solve": (ctypes.c_int, [CTX, ctypes.c_int, VP, VP, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
    "ibb_project": (ctypes.c_int, [CTX, VP, VP, VP]),
    "ibb_interp": (ctypes.c_int, [CTX, ctypes.c_double, I64, VP, VP, VP]),
    "ibb_spread": (ctypes.c_int, [CTX, ctypes.c_double, I64, VP, VP, VP]),
    "ibb_spread_static": (ctypes.c_int, [DESC, ctypes.c_double, I64, VP, VP, VP, VP]),
    "ibb_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ibb_last_error": (ctypes.c_char_p, [CTX]),
    "ibb_profile_enable": (ctypes.c_int, [CTX, ctypes.c_int]),
    "ibb_profile_read": (ctypes.c_int, [CTX, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]),
    "ibb_level_info": (ctypes.c_int, [CTX, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "ibb_fragments": (ctypes.c_int, [CTX, VP, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "ibb_group_footprint_bytes": (ctypes.c_int, [ctypes.POINTER(CTX), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "ibb_group_create": (ctypes.c_int, [ctypes.POINTER(CTX), ctypes.c_int, VP, ctypes.c_size_t,
                                        ctypes.POINTER(VP)]),
    "ibb_group_destroy": (ctypes.c_int, [VP]),
    "ibb_group_set_active": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int]),
    "ibb_group_projection_step": (ctypes.c_int, [VP, ctypes.POINTER(SolveStats)]),
    "ibb_group_lagrangian_update": (ctypes.c_int, [VP, ctypes.POINTER(LagStats)]),
    "ibb_group_last_error": (ctypes.c_char_p, [VP]),
}

_lib = None


def library_path():
    return os.path.join(HERE, "libibmg.so")


def load():
    """Load libibmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1302_3663_amd/build.py (no fallback exists)")
    # torch provides the device memory and streams, so the library must bind
    # to the HIP runtime torch loads; loaded before torch, the library would
    # bring in a second runtime, which then finds no device
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    for name, (res, args) in ABI_FUNCTIONS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L
