"""One time step of the method, in the order of the paper's "Solution
Strategy" section (TEST INFRASTRUCTURE ONLY).

    b_u   <- rho^n (sigma u^n / dt - N(u^n)) + C_f f^n + g        (eq:NSdis1-1)
    u~    <- MG(A_u(rho^n, mu^n), b_u, x0 = u^n)
    b_p   <- -(sigma / (eps dt)) D u~                              (eq:NSdis4)
    p     <- MG(A_p(1 / rho^n), b_p, x0 = p^n)
    u^n+1 <- u~ - (eps dt / sigma) beta G p                        (eq:NSdis2)
    U     <- J_h u^n+1 at X^n                                      (eq:discrVelCouple)
    X^n+1 <- X^n + (dt / sigma) U  (periodic axes wrap)
    springs: break those stretched past break_ratio x rest, then forces
    fragments: connected components of the alive springs (when tracked)
    f, rho, mu <- spread at X^n+1                                  (eq:discrForceCouple,
                                                                    eq:discrDensCouple, eq:ViscExp)
"""
import numpy as np

from . import (AX_INOUT, AX_PERIODIC, Hierarchy, anchored_nodes, density, fragments, interp_vec, momentum_rhs,
               pressure_rhs, project, spread_vec, springs, viscosity_cells, viscosity_edges)


class State:
    """Everything the step carries from one time level to the next."""

    def __init__(self, p, u, pres, X, ij, rest, K, alive=None):
        self.p = p
        self.u = np.array(u, dtype=np.float64)
        self.pres = np.array(pres, dtype=np.float64)
        self.X = np.array(X, dtype=np.float64)
        self.ij = np.array(ij, dtype=np.int32)
        self.rest = np.array(rest, dtype=np.float64)
        self.K = np.array(K, dtype=np.float64)
        self.alive = np.ones(self.ij.shape[1], np.uint8) if alive is None else np.array(alive, np.uint8)
        self.F = None
        self.f = self.rho = self.mu_c = self.mu_e = None
        self.hier = None
        self.step = 0
        self.anchored = anchored_nodes(p, self.X)   # at t = 0


def update_coefficients(st, do_break):
    """Forces at the current positions, then the Eulerian force, density and
    viscosity fields and the multigrid hierarchy built from them."""
    p = st.p
    st.F, st.alive, nb = springs(p, st.X, st.ij, st.rest, st.K, st.alive, do_break=do_break)
    st.f = spread_vec(p, p["omega"], st.X, st.F)
    st.rho = density(p, st.X)
    st.mu_c = viscosity_cells(p, st.X)
    st.mu_e = viscosity_edges(p, st.X)
    st.hier = Hierarchy(p, st.rho, st.mu_c, st.mu_e)
    return nb


def setup(st):
    return update_coefficients(st, do_break=False)


def pressure_singular(p):
    return all(p["axis_bc"][a] != AX_INOUT for a in range(p["dim"]))


def solve(st, velocity, b, x0):
    """Plain V-cycles, or V-cycle-preconditioned GCR(m) when krylov_restart = m > 0."""
    m = int(st.p.get("krylov_restart", 0))
    if m > 0:
        return st.hier.solve_gcr(velocity, b, x0, m=m)
    return st.hier.solve(velocity, b, x0)


def projection_step(st):
    """Momentum solve, pressure solve and projection (returns solve stats)."""
    p = st.p
    b_u = momentum_rhs(p, st.u, st.rho, st.mu_c, st.mu_e, st.f)
    ut, su = solve(st, True, b_u, st.u)
    b_p = pressure_rhs(p, ut)
    pres, sp = solve(st, False, b_p, st.pres)
    if pressure_singular(p):
        pres = pres - pres.mean()
    st.u = project(p, ut, pres, st.rho)
    st.pres = pres
    return dict(u=su, p=sp, b_u=b_u, b_p=b_p, ut=ut)


def wrap_positions(p, X):
    X = X.copy()
    for a in range(p["dim"]):
        if p["axis_bc"][a] == AX_PERIODIC:
            Lx = p["n"][a] * p["h"]
            X[a] = X[a] - Lx * np.floor(X[a] / Lx)
    return X


def lagrangian_update(st):
    """Interpolate, move the nodes, break and re-force the springs, spread."""
    p = st.p
    U = interp_vec(p, p["h"], st.X, st.u)
    st.X = wrap_positions(p, st.X + (p["dt"] / p["sigma"]) * U)
    nb = update_coefficients(st, do_break=True)
    st.step += 1
    out = dict(U=U, n_broken=nb, n_alive=int(st.alive.sum()))
    if p.get("track_fragments"):
        out["label"], out["n_fragments"], out["n_detached"] = fragments(st.ij, st.alive, st.anchored)
    return out


def run(st, steps):
    out = []
    for _ in range(steps):
        s = projection_step(st)
        l = lagrangian_update(st)
        out.append((s, l))
    return out
