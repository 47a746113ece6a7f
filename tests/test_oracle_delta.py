"""Pins for the regularised delta (Sec. "Dirac Delta Approximation").

Closed forms: phi(0) = 1/2 for both kernels, support |r| < 2, evenness, the
unity condition sum_j phi(r - j) = 1 for both kernels and the first-moment
condition sum_j (r - j) phi(r - j) = 0 for Peskin's kernel only
(eq:unityConditionDirac, eq:1stMomentConditionDirac with omega = h), the
textbook identity sum_j phi_1(r - j)^2 = 3/8 of Peskin's kernel, and the
paper's statements about the error metrics eq:PhiErrorUnity and
eq:PhiErrorFirstMomentum: both vanish for phi_1 when h = omega / z, and
phi_2 is the better choice at the paper's omega = 1/100, h = 1/128.
"""
import numpy as np
import pytest

import oracle as O

COS, PESKIN = 0, 1


@pytest.mark.parametrize("k", [COS, PESKIN])
def test_phi_centre_support_even(k):
    assert O.phi(k, 0.0)[0] == 0.5
    r = np.linspace(-3, 3, 601)
    v = O.phi(k, r)
    assert np.all(v[np.abs(r) >= 2.0] == 0.0)
    assert np.all(v[np.abs(r) < 2.0] > 0.0)
    np.testing.assert_array_equal(v, O.phi(k, -r))


def test_peskin_branches_meet():
    # both branches of eq:PhiPeskin give 1/4 at |r| = 1
    a = O.phi(PESKIN, 1.0 - 1e-12)[0]
    b = O.phi(PESKIN, 1.0 + 1e-12)[0]
    assert abs(a - 0.25) < 1e-9 and abs(b - 0.25) < 1e-9


def test_cosine_closed_form_points():
    # phi_2(1) = 1/4 (cos(pi/2) = 0); phi_2(2/3) = (1 + cos(pi/3)) / 4 = 3/8
    assert abs(O.phi(COS, 1.0)[0] - 0.25) < 1e-15
    assert abs(O.phi(COS, 2.0 / 3.0)[0] - 0.375) < 1e-15


@pytest.mark.parametrize("k", [COS, PESKIN])
def test_unity_condition_at_omega_equal_h(k):
    for r in np.linspace(0.0, 1.0, 41):
        j = np.arange(-3, 5)
        assert abs(O.phi(k, r - j).sum() - 1.0) < 1e-14


def test_first_moment_peskin_only():
    j = np.arange(-3, 5)
    worst_cos = 0.0
    for r in np.linspace(0.0, 1.0, 41):
        m1 = ((r - j) * O.phi(PESKIN, r - j)).sum()
        assert abs(m1) < 1e-14
        worst_cos = max(worst_cos, abs(((r - j) * O.phi(COS, r - j)).sum()))
    assert worst_cos > 1e-4


def test_peskin_sum_of_squares():
    j = np.arange(-3, 5)
    for r in np.linspace(0.0, 1.0, 21):
        assert abs((O.phi(PESKIN, r - j) ** 2).sum() - 0.375) < 1e-14


def eps_metrics(k, omega, h, nx=2001):
    """eq:PhiErrorUnity and eq:PhiErrorFirstMomentum, 1D, X scanned over [0, h]."""
    m = int(np.ceil(2 * omega / h)) + 2
    x = np.arange(-m, m + 1) * h
    eu = em = 0.0
    for X in np.linspace(0.0, h, nx):
        w = O.phi(k, (x - X) / omega) / omega * h
        eu = max(eu, abs(w.sum() - 1.0))
        em = max(em, abs(((x - X) * w).sum()))
    return eu, em


@pytest.mark.parametrize("z", [1, 2, 4])
def test_peskin_exact_when_h_divides_omega(z):
    omega = 1.0 / 100
    eu, em = eps_metrics(PESKIN, omega, omega / z, nx=201)
    assert eu < 1e-13 and em < 1e-15


def test_cosine_wins_at_paper_resolution():
    # omega = 1/100 with h = 1/128 (the paper's simulations) favours phi_2
    eu1, _ = eps_metrics(PESKIN, 0.01, 1.0 / 128, nx=801)
    eu2, _ = eps_metrics(COS, 0.01, 1.0 / 128, nx=801)
    assert eu2 < eu1


def test_moment_errors_vanish_faster_than_h2():
    # as h -> 0 the defects fall at least like a Riemann sum, O(h^2) or faster
    e_a = eps_metrics(COS, 0.01, 1.0 / 128, nx=801)[0]
    e_b = eps_metrics(COS, 0.01, 1.0 / 1024, nx=201)[0]
    assert e_b / e_a < (128.0 / 1024.0) ** 2
