"""Helpers for the manufactured-solution pins: lattice coordinates of the
MAC positions and evaluation of sympy expressions on them.

Every lattice position (i, j, k) sits at x_d = i_d h along an axis where the
lattice is vertex-centred (faces normal to d, edges not parallel to d) and at
(i_d + 1/2) h along the others (cell centres).
"""
import numpy as np
import sympy as sp

import oracle as O

X, Y, Z = sp.symbols("x y z")
SYMS = (X, Y, Z)


def coords_of(p, kind, axis, q):
    """coordinates of lattice index rows q (n x 3)"""
    h = p["h"]
    out = np.zeros((q.shape[0], p["dim"]))
    for d in range(p["dim"]):
        vert = (kind == O.FACE and d == axis) or (kind == O.EDGE and d != axis)
        out[:, d] = q[:, d] * h if vert else (q[:, d] + 0.5) * h
    return out


def lattice_index(p, kind, axis):
    """index rows of every stored position of a lattice, compact order"""
    _, dims = O.lattice_dims(p, kind, axis)
    k, j, i = np.meshgrid(np.arange(dims[2]), np.arange(dims[1]), np.arange(dims[0]), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def all_points(p, kind, axis):
    return coords_of(p, kind, axis, lattice_index(p, kind, axis))


def evaluate(expr, pts):
    """a sympy expression in x, y (, z) at the rows of pts"""
    D = pts.shape[1]
    f = sp.lambdify(SYMS[:D], expr, "numpy")
    v = f(*[pts[:, d] for d in range(D)])
    return np.broadcast_to(np.asarray(v, dtype=float), (pts.shape[0],)).copy()


def edge_axes(p):
    return [0, 1, 2] if p["dim"] == 3 else [2]


def faces(p, exprs):
    """compact face field: component a of exprs on the a-faces"""
    return np.concatenate([evaluate(exprs[a], all_points(p, O.FACE, a)) for a in range(p["dim"])])


def face_scalar(p, expr):
    """compact face field: one scalar expression on every face lattice"""
    return faces(p, [expr] * p["dim"])


def cells(p, expr):
    return evaluate(expr, all_points(p, O.CELL, 0))


def edges(p, expr):
    return np.concatenate([evaluate(expr, all_points(p, O.EDGE, c)) for c in edge_axes(p)])


def gather(p, compact_faces, comp, pos):
    """values of a compact face field at the unknown rows (comp, pos)"""
    f = O.split_faces(p, compact_faces)
    out = np.zeros(comp.size)
    for a in range(p["dim"]):
        s = comp == a
        q = pos[s]
        out[s] = f[a][q[:, 2], q[:, 1], q[:, 0]]
    return out


def scatter(p, values, comp, pos):
    """compact face field holding `values` at the unknown rows, 0 elsewhere"""
    f = O.split_faces(p, np.zeros(sum(O.face_counts(p))))
    for a in range(p["dim"]):
        s = comp == a
        q = pos[s]
        f[a][q[:, 2], q[:, 1], q[:, 0]] = values[s]
    return np.concatenate([v.ravel() for v in f])
