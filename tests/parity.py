"""Parity metrics shared by the GPU tests: relative difference of two fields
in the 2-norm and in the max norm (||a - b|| / ||b||, both per field).  A
field passes only when both are within the tolerance, so a single point off
among millions is not hidden by the 2-norm."""
import numpy as np


def rel2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def relinf(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    nb = np.abs(b).max()
    return np.abs(a - b).max() / (nb if nb > 0 else 1.0)


def close(a, b, tol):
    """True when a matches b within tol in both norms."""
    return rel2(a, b) < tol and relinf(a, b) < tol


def check(a, b, tol, what=""):
    r2, ri = rel2(a, b), relinf(a, b)
    assert r2 < tol and ri < tol, f"{what}: rel 2-norm {r2:.3e}, max norm {ri:.3e}, tolerance {tol:.0e}"


def rel(a, b):
    """the larger of the relative 2-norm and max-norm differences"""
    return max(rel2(a, b), relinf(a, b))
