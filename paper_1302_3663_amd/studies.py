"""Empirical convergence rates of the whole time step, the refinement studies
of the paper's validation section, run through the library.

Temporal (eq:ErrorTemporal, eq:temporal convergence rate): the same grid and
nodes stepped to time T with dt, dt/2, dt/4, ...; the error of a run is its
distance at T from the run with half its step, and the rate is log2 of the
ratio of consecutive errors.

Spatial (eq:ErrorSpatial, eq:convergenceRate): the same nodes on grids of
width h, h/2, h/4, ... at a fixed step; the velocity error of a grid is its
distance from the full-weighting restriction of the next finer grid's
velocity, the node error the plain distance of the node positions.

Norms: max norm, and the discrete 2-norm scaled by the cell volume (velocity)
or by the node count (positions).  First-order rates are what the paper
reports and expects for an interface that is not smooth.

The studies here use the 2D channel (periodic in x, walls in y) of the
workloads; every time step runs on the GPU, and only the error norms and the
restriction that compares two grids are host arithmetic.

    python -m paper_1302_3663_amd.studies [--out FILE]
"""
import argparse
import json
import math

import numpy as np

from . import synth

AX_PERIODIC, AX_WALLS = synth.AX_PERIODIC, synth.AX_WALLS


def run_to(case, dt, T, precision=0, inner_cycles=2):
    """Step `case` with step dt until time T; -> (velocity faces, nodes).
    The case's own parameters choose the solver (e.g. krylov_restart)."""
    from . import ibmg
    steps = int(round(T / dt))
    if abs(steps * dt - T) > 1e-9 * T:
        raise ValueError(f"T = {T} is not a whole number of steps of {dt}")
    c = dict(case, params=dict(case["params"], dt=dt))
    ctx = ibmg.from_case(c, precision=precision, inner_cycles=inner_cycles)
    try:
        for _ in range(steps):
            ctx.projection_step()
            ctx.lagrangian_update()
        u, _ = ctx.get_state()
        X, _, _ = ctx.get_nodes()
        import torch
        torch.cuda.synchronize()
        return u.cpu().numpy().copy(), X.cpu().numpy().copy()
    finally:
        ctx.close()


def split_faces_2d(p, u):
    """Compact face vector -> [x-face array (ny, nx_x), y-face array (ny_y, nx)]."""
    out, off = [], 0
    for a in range(2):
        dims = synth.face_dims(p, a)
        n = dims[0] * dims[1]
        out.append(u[off:off + n].reshape(dims[1], dims[0]))
        off += n
    return out


def _axis_weights(vertex):
    # full weighting along one axis (coarse index I): fine offsets and weights
    if vertex:
        return [(-1, 0.25), (0, 0.5), (1, 0.25)]
    return [(-1, 0.125), (0, 0.375), (1, 0.375), (2, 0.125)]


def restrict_channel_faces(p_fine, u_fine):
    """Full weighting of the velocity of the 2D channel from a grid to the
    grid of twice the width: per axis (1/4, 1/2, 1/4) along the face normal
    and (1/8, 3/8, 3/8, 1/8) across it.  x is periodic; across the walls the
    tangential velocity reflects oddly (zero on the wall) and wall-normal
    faces hold zero."""
    if p_fine["dim"] != 2 or p_fine["axis_bc"][0] != AX_PERIODIC or p_fine["axis_bc"][1] != AX_WALLS:
        raise ValueError("restrict_channel_faces expects the 2D channel (periodic x, walls in y)")
    nx, ny = p_fine["n"][0], p_fine["n"][1]
    fx, fy = split_faces_2d(p_fine, u_fine)
    cx, cy = nx // 2, ny // 2
    # x-faces: vertex along x (periodic, nx faces), cell along y (ny cells, odd at the walls)
    ux = np.zeros((cy, cx))
    for J in range(cy):
        for I in range(cx):
            s = 0.0
            for dj, wj in _axis_weights(False):
                j = 2 * J + dj
                sign = 1.0
                if j < 0:
                    j, sign = -1 - j, -1.0
                elif j >= ny:
                    j, sign = 2 * ny - 1 - j, -1.0
                for di, wi in _axis_weights(True):
                    i = (2 * I + di) % nx
                    s += wi * wj * sign * fx[j, i]
            ux[J, I] = s
    # y-faces: vertex along y (walls: faces 0 and ny fixed at zero), cell along x (periodic)
    uy = np.zeros((cy + 1, cx))
    for J in range(1, cy):
        for I in range(cx):
            s = 0.0
            for dj, wj in _axis_weights(True):
                j = 2 * J + dj
                for di, wi in _axis_weights(False):
                    i = (2 * I + di) % nx
                    s += wi * wj * fy[j, i]
            uy[J, I] = s
    return np.concatenate([ux.ravel(), uy.ravel()])


def _norms_u(e, h, dim=2):
    return float(np.max(np.abs(e))), float(math.sqrt(h ** dim * np.sum(e * e)))


def _norms_x(e):
    d = e.reshape(e.shape[0], -1)
    return float(np.max(np.abs(d))), float(math.sqrt(np.sum(d * d) / d.shape[1]))


def rates(errors):
    """log2 of consecutive error ratios."""
    return [math.log2(a / b) if a > 0 and b > 0 else float("nan") for a, b in zip(errors, errors[1:])]


def temporal_study(case, dts, T, precision=0):
    """Errors E(q(T); dt) for dt in dts (each halving the previous; the last
    run only serves as the reference of the one before) and their rates."""
    runs = [run_to(case, dt, T, precision) for dt in dts]
    h = case["params"]["h"]
    out = {"dt": list(dts[:-1]), "u_inf": [], "u_2": [], "X_inf": [], "X_2": []}
    for (ua, Xa), (ub, Xb) in zip(runs, runs[1:]):
        ui, u2 = _norms_u(ua - ub, h, case["params"]["dim"])
        xi, x2 = _norms_x(Xa - Xb)
        out["u_inf"].append(ui)
        out["u_2"].append(u2)
        out["X_inf"].append(xi)
        out["X_2"].append(x2)
    for q in ("u_inf", "u_2", "X_inf", "X_2"):
        out["rate_" + q] = rates(out[q])
    return out


def spatial_study(make_case, ns, dt, T, precision=0):
    """make_case(ny) -> channel case with ny cells across (same nodes for
    every ny); errors E(q(T); h) for consecutive refinements and rates."""
    runs = []
    for ny in ns:
        case = make_case(ny)
        runs.append((case["params"], run_to(case, dt, T, precision)))
    out = {"h": [], "u_inf": [], "u_2": [], "X_inf": [], "X_2": []}
    for (pa, (ua, Xa)), (pb, (ub, Xb)) in zip(runs, runs[1:]):
        ui, u2 = _norms_u(ua - restrict_channel_faces(pb, ub), pa["h"])
        xi, x2 = _norms_x(Xa - Xb)
        out["h"].append(pa["h"])
        out["u_inf"].append(ui)
        out["u_2"].append(u2)
        out["X_inf"].append(xi)
        out["X_2"].append(x2)
    for q in ("u_inf", "u_2", "X_inf", "X_2"):
        out["rate_" + q] = rates(out[q])
    return out


def channel(ny, seed=1, eta=30, mu_max=1.0, rho_b=0.0, krylov=0):
    """The 2D channel of the workloads ([0,2] x [0,1], nodes uniform in a
    half-disc of radius 0.25 on the bottom wall, springs of stiffness 1e2
    within 0.08) on a grid with ny cells across; the nodes do not depend on
    ny.  As in the paper's studies the default biofilm has the fluid's
    density and viscosity.  No spring breaks within the studied time (a break
    is an event, not a smooth function of the step)."""
    case = synth.channel_2d(seed=seed, nx=2 * ny, ny=ny, eta=eta)
    case["params"].update(mu_max=mu_max, rho_b=rho_b, break_ratio=100.0, krylov_restart=krylov)
    return case


STUDIES = {
    # name: (kind, case (temporal) or case maker of ny (spatial), refinements)
    "temporal": ("temporal", lambda: channel(32), [4e-4, 2e-4, 1e-4, 5e-5, 2.5e-5]),
    "temporal_200_nodes": ("temporal", lambda: channel(32, eta=200), [4e-4, 2e-4, 1e-4, 5e-5, 2.5e-5]),
    "spatial": ("spatial", channel, [32, 64, 128, 256, 512]),
    "spatial_density2": ("spatial", lambda ny: channel(ny, rho_b=1.0), [32, 64, 128, 256, 512]),
    "spatial_viscosity500": ("spatial", lambda ny: channel(ny, mu_max=500.0, krylov=8), [32, 64, 128, 256, 512]),
}


def run_study(name, T=3.2e-3, dt=1e-4):
    kind, make, refs = STUDIES[name]
    if kind == "temporal":
        return temporal_study(make(), refs, T)
    return spatial_study(make, refs, dt, T)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=None)
    ap.add_argument("--T", type=float, default=3.2e-3)
    ap.add_argument("--only", default=None, help="comma-separated study names")
    args = ap.parse_args()
    names = args.only.split(",") if args.only else list(STUDIES)
    res = {n: run_study(n, args.T) for n in names}
    text = json.dumps(res, indent=1)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()
