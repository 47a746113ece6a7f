"""The delta-kernel error metrics eq:PhiErrorUnity and eq:PhiErrorFirstMomentum
measured through the GPU spread (studies.delta_errors) against the 1D sums of
the oracle's phi at the same node offsets, for both kernels; phi_1 is exact
when the mesh width divides the spread width."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1302_3663_amd import studies

pytestmark = pytest.mark.gpu


def oracle_1d(kernel, omega, h, ts):
    m = int(math.ceil(2 * omega / h)) + 2
    x = np.arange(-m, m + 1) * h
    su, mo = [], []
    for t in ts:
        w = O.phi(kernel, (x - t) / omega) / omega * h
        su.append(w.sum() - 1.0)
        mo.append(((x - t) * w).sum())
    return np.array(su), np.array(mo)


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("h", [0.01 / 4, 1.0 / 128, 1.0 / 1000])
def test_gpu_metrics_match_oracle(kernel, h):
    omega, nsamp = 0.01, 9
    g = studies.delta_errors(kernel, omega, h, nsamp)
    su, mo = oracle_1d(kernel, omega, h, np.linspace(0.0, h, nsamp))
    print(kernel, h, g["eps_unity"], g["eps_mom"], flush=True)
    assert np.max(np.abs(np.array(g["unity"]) - su)) < 1e-13
    assert np.max(np.abs(np.array(g["moment"]) - mo)) < 1e-13 * omega


def test_phi1_exact_at_divisors():
    for z in (1, 2, 5):
        g = studies.delta_errors(1, 0.01, 0.01 / z, 9)
        assert g["eps_unity"] < 1e-13 and g["eps_mom"] < 1e-15
