"""The hovering insect's prescribed wing motion (Sec. 3: alpha(t) = alpha0 [1 + sin(2 pi f t)],
wings hinged at the body and flapping symmetrically), checked against geometry and calculus
rather than against the formula: the wings stay rigid, each wing's root vertex stays at its
hinge, the flapping angle spans [0, 2 alpha0] with the stroke's extremes at the quarter
periods, the wings mirror each other, the body does not move, the velocities are the time
derivatives of the positions, and the wing weights add up to the ellipse's perimeter."""
import math

import numpy as np
import pytest
from scipy.special import ellipe

from paper_1905_00182_amd import workloads as W


@pytest.fixture(scope="module")
def case():
    return W.insect(n=192, L=3.84, sponge=0.5, nprobe=0)


def _parts(case, A):
    nb = len(case.extra["insect"]["body_x"])
    nw = len(case.extra["insect"]["theta"])
    return A[:, :nb], A[:, nb:nb + nw], A[:, nb + nw:]


def _axis_angle(case, wing):
    # centre and major axis from the markers' first and second moments: at equal parameter
    # steps the mean is the centre and the covariance is diag(a^2/2, b^2/2) in the wing frame
    c = wing.mean(axis=1)
    w, v = np.linalg.eigh(np.cov(wing, bias=True))
    ax = v[:, np.argmax(w)]
    if ax[0] < 0:
        ax = -ax                 # pointing away from the hinge (|alpha| < 90 degrees)
    return c, math.atan2(ax[1], ax[0])


def test_rigid_wings_and_static_body(case):
    X0, _ = W.insect_kinematics(case, 0.0)
    b0, r0, _ = _parts(case, X0)
    for t in (3.1, 11.0, 27.7):
        X, U = W.insect_kinematics(case, t)
        b, r, _ = _parts(case, X)
        np.testing.assert_array_equal(b, b0)
        assert np.all(_parts(case, U)[0] == 0.0)
        d0 = np.hypot(*(r0[:, :, None] - r0[:, None, :]))
        d = np.hypot(*(r[:, :, None] - r[:, None, :]))
        np.testing.assert_allclose(d, d0, atol=1e-14)


def test_root_at_the_hinge_and_flapping_angle(case):
    p = case.extra["insect"]
    T = 1.0 / p["f"]
    for t, alpha in ((0.0, p["alpha0"]), (0.25 * T, 2 * p["alpha0"]), (0.75 * T, 0.0), (0.5 * T, p["alpha0"])):
        X, _ = W.insect_kinematics(case, t)
        _, r, _ = _parts(case, X)
        c, ang = _axis_angle(case, r)
        root = c - p["a"] * np.array([math.cos(ang), math.sin(ang)])
        np.testing.assert_allclose(root, [p["hinge"], 0.0], atol=1e-13)
        assert ang == pytest.approx(alpha, abs=1e-13)
    assert p["alpha0"] == pytest.approx(math.radians(25.3))


def test_wings_mirror_each_other(case):
    for t in (0.0, 7.9, 21.3):
        X, U = W.insect_kinematics(case, t)
        _, r, l = _parts(case, X)
        _, ur, ul = _parts(case, U)
        np.testing.assert_array_equal(l, r * np.array([[-1.0], [1.0]]))
        np.testing.assert_array_equal(ul, ur * np.array([[-1.0], [1.0]]))


def test_velocities_are_time_derivatives(case):
    for t in (0.0, 5.3, 33.3):
        e = 1e-4
        Xp, _ = W.insect_kinematics(case, t + e)
        Xm, _ = W.insect_kinematics(case, t - e)
        _, U = W.insect_kinematics(case, t)
        np.testing.assert_allclose(U, (Xp - Xm) / (2 * e), atol=1e-9)
        assert np.abs(U).max() > 1e-3


def test_wing_weights_add_up_to_the_perimeter(case):
    p = case.extra["insect"]
    nb, nw = len(p["body_x"]), len(p["theta"])
    dV = case.markers["dV"]
    a, b = p["a"], p["b"]
    perim = 4 * a * ellipe(1 - (b / a) ** 2)          # complete elliptic integral of the second kind
    assert dV[nb:nb + nw].sum() == pytest.approx(perim, rel=1e-12)
    assert dV[:nb].sum() == pytest.approx(2 * math.pi * p["hinge"], rel=1e-14)
