"""The rigid flapping plate's prescribed kinematics (Sec. 4.1: the clamped leading edge moves as
X0(t) = (A0/2) cos(2 pi f t) [cos beta, sin beta] and pitches by alpha(t) = (alpha_m/2)
sin(2 pi f t + phi)), checked against geometry and calculus rather than against the formula:
the plate stays rigid, its leading edge passes through the stroke's turning points and centre
at the quarter periods, its slope at a quarter period is the pitch amplitude, and the marker
velocities are the time derivatives of the positions.  Also: the oracle's kinematics update
keeps the penalty integral."""
import math

import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W


@pytest.fixture(scope="module")
def case():
    return W.config5(n=128, L=8.0, nmark=64)


def _edge(case, t):
    # the leading edge by linear extrapolation of the first two markers to s = 0
    X, _ = W.plate_kinematics(case, t)
    s = case.extra["plate"]["s"]
    return X[:, 0] - s[0] * (X[:, 1] - X[:, 0]) / (s[1] - s[0])


def test_rigid_plate(case):
    ds = 1.0 / 64
    for t in (0.0, 3.7, 19.6, 41.2):
        X, _ = W.plate_kinematics(case, t)
        gaps = np.hypot(*np.diff(X, axis=1))
        np.testing.assert_allclose(gaps, ds, rtol=1e-12)


def test_leading_edge_stroke(case):
    T = 1.0 / case.extra["plate"]["f"]
    x_edge = case.extra["plate"]["edge"][0]
    np.testing.assert_allclose(_edge(case, 0.0), [x_edge, 0.5], atol=1e-12)        # top of the stroke
    np.testing.assert_allclose(_edge(case, 0.25 * T), [x_edge, 0.0], atol=1e-12)   # centre, moving down
    np.testing.assert_allclose(_edge(case, 0.5 * T), [x_edge, -0.5], atol=1e-12)   # bottom
    np.testing.assert_allclose(_edge(case, T), [x_edge, 0.5], atol=1e-12)          # one period


def test_pitch_amplitude(case):
    T = 1.0 / case.extra["plate"]["f"]
    X, _ = W.plate_kinematics(case, 0.25 * T)
    slope = (X[1, -1] - X[1, 0]) / (X[0, -1] - X[0, 0])
    assert slope == pytest.approx(-math.tan(math.radians(30.0)), rel=1e-12)   # nose up by 30 degrees
    X, _ = W.plate_kinematics(case, 0.0)
    assert np.ptp(X[1]) == 0.0                                                 # level at t = 0


def test_velocities_are_time_derivatives(case):
    for t in (0.0, 7.3, 30.1):
        e = 1e-3
        Xp, _ = W.plate_kinematics(case, t + e)
        Xm, _ = W.plate_kinematics(case, t - e)
        _, U = W.plate_kinematics(case, t)
        np.testing.assert_allclose(U, (Xp - Xm) / (2 * e), atol=1e-9)
        assert np.abs(U).max() > 1e-3


def test_oracle_kinematics_keep_the_integral(case):
    from oracle.oracle import Oracle

    o = Oracle(case)
    xi = np.arange(2 * 64, dtype=np.float64).reshape(2, 64) * 1e-3
    o.set_state(xi, 1.5, 7)
    X, U = W.plate_kinematics(case, 1.5)
    o.set_marker_kinematics(X, U)
    xg, t, step = o.get_state()
    np.testing.assert_array_equal(xg, xi)
    assert (t, step) == (1.5, 7)
