"""The refinement studies on the GPU (paper_1302_3663_amd.studies): the
temporal study's errors equal the oracle's on the same runs, and converge at
first order for the coarser steps; the spatial study converges at first
order or better in the 2-norms of velocity and node positions once the
spread width exceeds the mesh width."""
import numpy as np
import pytest

from oracle import step as S
from paper_1302_3663_amd import studies

pytestmark = pytest.mark.gpu


def oracle_temporal_errors(case, dts, T):
    runs = []
    for dt in dts:
        p = dict(case["params"], dt=dt)
        st = S.State(p, case["u0"], case["p0"], case["X"], case["ij"], case["rest"], case["K"])
        S.setup(st)
        for _ in range(int(round(T / dt))):
            S.projection_step(st)
            S.lagrangian_update(st)
        runs.append((st.u.copy(), st.X.copy()))
    eu = [float(np.max(np.abs(a[0] - b[0]))) for a, b in zip(runs, runs[1:])]
    ex = [float(np.max(np.abs(a[1] - b[1]))) for a, b in zip(runs, runs[1:])]
    return eu, ex


def test_temporal_matches_oracle_and_is_first_order():
    case = studies.channel(32)
    dts = [4e-4, 2e-4, 1e-4]
    g = studies.temporal_study(case, dts, 3.2e-3)
    eu, ex = oracle_temporal_errors(case, dts, 3.2e-3)
    print("gpu", g["u_inf"], g["X_inf"], "oracle", eu, ex, flush=True)
    assert np.allclose(g["u_inf"], eu, rtol=1e-6, atol=0)
    assert np.allclose(g["X_inf"], ex, rtol=1e-6, atol=0)
    for q in ("u_inf", "X_inf"):
        assert 0.75 < g["rate_" + q][0] < 1.25


def test_spatial_first_order_or_better():
    r = studies.spatial_study(studies.channel, [32, 64, 128], 1e-4, 3.2e-3)
    print(r, flush=True)
    for q in ("u_2", "X_2", "X_inf"):
        assert r["rate_" + q][0] > 0.9, (q, r["rate_" + q])
