"""The refinement studies of the validation section (eq:ErrorTemporal,
eq:ErrorSpatial) on the CPU:
- the full-weighting restriction used to compare two grids' velocities is
  second-order accurate on smooth fields that obey the channel's boundary
  conditions;
- the oracle's time step converges at first order in time on the channel
  with a uniform biofilm (the paper's expectation for a non-smooth
  interface), for the coarser steps of the study."""
import math

import numpy as np
import pytest

from oracle import step as S
from paper_1302_3663_amd import studies, synth


def channel_field(ny):
    p = synth.channel_2d(nx=2 * ny, ny=ny, eta=10)["params"]
    h, nx = p["h"], 2 * ny
    x_face, y_cell = np.arange(nx) * h, (np.arange(ny) + 0.5) * h
    ux = np.sin(math.pi * y_cell)[:, None] * np.cos(math.pi * x_face)[None, :]
    x_cell, y_face = (np.arange(nx) + 0.5) * h, np.arange(ny + 1) * h
    uy = np.sin(math.pi * y_face)[:, None] * np.sin(math.pi * x_cell)[None, :]
    return p, np.concatenate([ux.ravel(), uy.ravel()])


def test_restriction_is_second_order():
    errs = []
    for ny in (8, 16, 32):
        pf, uf = channel_field(2 * ny)
        _, uc = channel_field(ny)
        errs.append(np.max(np.abs(studies.restrict_channel_faces(pf, uf) - uc)))
    r = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(1.9 < x < 2.1 for x in r), r


def oracle_run(case, dt, T):
    p = dict(case["params"], dt=dt)
    st = S.State(p, case["u0"], case["p0"], case["X"], case["ij"], case["rest"], case["K"])
    S.setup(st)
    for _ in range(int(round(T / dt))):
        S.projection_step(st)
        S.lagrangian_update(st)
    return st.u.copy(), st.X.copy()


def oracle_temporal_errors(case, dts, T):
    runs = [oracle_run(case, dt, T) for dt in dts]
    eu = [float(np.max(np.abs(a[0] - b[0]))) for a, b in zip(runs, runs[1:])]
    ex = [float(np.max(np.abs(a[1] - b[1]))) for a, b in zip(runs, runs[1:])]
    return eu, ex


def test_oracle_first_order_in_time():
    eu, ex = oracle_temporal_errors(studies.channel(32), [4e-4, 2e-4, 1e-4], 3.2e-3)
    for e in (eu, ex):
        r = math.log2(e[0] / e[1])
        assert 0.75 < r < 1.25, (e, r)
