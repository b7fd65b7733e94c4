"""Pins of the oracle's periodic Gaussian pressure source (Sec. 3, scattering by a stationary
sphere: A_p = -A exp(-B log(2) r^2) cos(omega t), read as the energy source A_p / (gamma - 1))
against facts that do not come from its own formula: the half-width meaning of B log 2 on
cells at known distances, the sign and size at the centre, the period of cos, the closed-form
Gaussian integral, and SSP-RK3's stage times (for a source that depends on t alone, one step
adds dt times Simpson's rule of the source over the step)."""
import math

import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

GM1 = W.GAMMA - 1.0


def _oracle(case):
    from oracle.oracle import Oracle

    return Oracle(case)


def _box(n, h, centre, amp=0.01, b=16.0, omega=2.0 * math.pi):
    # only the source: no convection, viscosity, sponge or markers
    return W.periodic_box(dim=3, n=n, L=n * h).with_(terms=0, src_amp=amp, src_b=b, src_omega=omega,
                                                     src_x=centre)


def _energy_rhs(case, t):
    o = _oracle(case)
    o.set_state(None, t, 0)
    L = o.rhs(W.uniform_state(case))
    assert np.all(L[:4] == 0.0)
    return L[4]


def test_centre_and_half_width():
    # centre on cell (8, 8, 8) of a 0.25 grid; B = 16 puts half the peak at r = 1/4
    h = 0.25
    case = _box(16, h, centre=(8.5 * h, 8.5 * h, 8.5 * h))
    E = _energy_rhs(case, 0.0)
    peak = E[8, 8, 8]
    assert peak == pytest.approx(-0.01 / GM1, rel=1e-15)
    assert E[8, 8, 9] == pytest.approx(peak / 2, rel=1e-14)     # face neighbour, r^2 = h^2
    assert E[8, 9, 9] == pytest.approx(peak / 4, rel=1e-14)     # edge neighbour, r^2 = 2 h^2
    assert E[9, 9, 9] == pytest.approx(peak / 8, rel=1e-14)     # corner neighbour, r^2 = 3 h^2
    assert E[7, 8, 8] == E[9, 8, 8] == E[8, 7, 8] == E[8, 8, 7]  # isotropic
    assert np.all(E < 0.0) and E.min() == peak


def test_period_and_sign_in_time():
    case = _box(12, 0.25, centre=(1.3, 1.6, 1.45))
    E0 = _energy_rhs(case, 0.0)
    np.testing.assert_array_equal(_energy_rhs(case, 0.5), -E0)   # omega t = pi
    np.testing.assert_array_equal(_energy_rhs(case, 1.0), E0)    # a whole period
    assert np.abs(_energy_rhs(case, 0.25)).max() < 1e-15 * np.abs(E0).max()   # omega t = pi/2


def test_gaussian_integral_closed_form():
    # the midpoint sum of a Gaussian this well resolved equals its integral to rounding:
    # sum_cells A_p h^3 = -A (pi / (B log 2))^(3/2)
    h = 0.125
    case = _box(64, h, centre=(4.03, 3.97, 4.11))
    E = _energy_rhs(case, 0.0)
    total = E.sum() * h**3 * GM1
    exact = -0.01 * (math.pi / (16.0 * math.log(2.0))) ** 1.5
    assert total == pytest.approx(exact, rel=1e-12)


def test_rk3_stage_times_simpson():
    # y' = F(t): SSP-RK3 gives y1 - y0 = dt (F(t0) + F(t0 + dt) + 4 F(t0 + dt/2)) / 6
    case = _box(8, 0.25, centre=(1.0, 1.0, 1.0))
    t0, dt = 0.3, 0.1
    F = [_energy_rhs(case, t) for t in (t0, t0 + dt, t0 + 0.5 * dt)]
    o = _oracle(case)
    o.set_state(None, t0, 0)
    Q0 = W.uniform_state(case)
    Q = o.rk3_step(Q0.copy(), dt)
    np.testing.assert_array_equal(Q[:4], Q0[:4])
    expect = dt * (F[0] + F[1] + 4.0 * F[2]) / 6.0
    # (absolute part: a few ulps of E itself, which the stage combinations round)
    np.testing.assert_allclose(Q[4] - Q0[4], expect, rtol=1e-12, atol=8.0 * np.spacing(Q0[4].max()))
    # a wrong stage time would show: the midpoint weight is the large one
    assert np.abs(F[2] - F[1]).max() > 1e-3 * np.abs(F[2]).max()
