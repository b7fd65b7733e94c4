"""Pins of the oracle's flexible plate (absolute nodal coordinates, Sec. 2's beam equation)
against facts that do not come from its own formulas: the Euler-Bernoulli cantilever under a
uniform load (cubic Hermite elements reproduce its nodal deflections and slopes exactly), the
cantilever's natural frequencies (roots of 1 + cos x cosh x = 0), the total mass, the force
of a uniformly stretched plate (tension at the ends only, rotating with the plate), Newmark's
average-acceleration phase error on a single mode (amplitude kept, frequency
2 atan(w dt / 2) / dt), rigid transport at constant velocity, and the straight plate's
markers against the rigid plate's kinematics."""
import math

import numpy as np
import pytest
from scipy.linalg import eigh
from scipy.optimize import brentq

from oracle.ancf import Plate, flapping_clamp
from paper_1905_00182_amd import workloads as W

L, NEL, RHO, KS, KB = 1.0, 40, 5.0, 10.0, 0.01


def _rest(t):
    z = np.zeros(2)
    return z, np.array([1.0, 0.0]), z, z, z, z


def _plate(clamp=_rest, s_mark=None, dv=None, **kw):
    if s_mark is None:
        s_mark = (np.arange(64) + 0.5) / 64
        dv = np.full(64, 1.0 / 64)
    args = dict(length=L, nel=NEL, rho_s=RHO, k_s=KS, k_b=KB)
    args.update(kw)
    return Plate(s_mark=s_mark, dv_mark=dv, clamp=clamp, **args)


def _gauss_markers(nel=NEL, npt=3):
    # markers at Gauss points of every element: the load integral of a cubic is then exact
    x, w = np.polynomial.legendre.leggauss(npt)
    l = L / nel
    s = np.concatenate([j * l + 0.5 * l * (x + 1) for j in range(nel)])
    return s, np.tile(0.5 * l * w, nel)


def _yfree(nel):
    # free transverse coordinates of a plate along x (y position and y slope of nodes 1..nel)
    return np.array([i for i in range(4, 4 * (nel + 1)) if i % 4 in (1, 3)])


YF = _yfree(NEL)


def test_total_mass():
    p = _plate()
    tx = np.zeros(p.ndof)
    tx[0::4] = 1.0
    ty = np.zeros(p.ndof)
    ty[1::4] = 1.0
    assert tx @ p.M @ tx == pytest.approx(RHO * L, rel=1e-14)
    assert ty @ p.M @ ty == pytest.approx(RHO * L, rel=1e-14)
    assert abs(tx @ p.M @ ty) < 1e-15


@pytest.mark.parametrize("nel,rtol", [(4, 1e-13), (40, 1e-8)])
def test_cantilever_uniform_load_nodal_exact(nel, rtol):
    # (the tolerance is the static solve's rounding: the bending matrix's condition number,
    # 6.9e3 at 4 elements and 6.1e7 at 40, times the unit roundoff)
    s, dv = _gauss_markers(nel)
    q = 1e-3
    p = _plate(s_mark=s, dv=dv, nel=nel)
    F = np.zeros((2, len(s)))
    F[1] = q
    Q = p.load(F)
    assert Q[1::4].sum() == pytest.approx(q * L, rel=1e-14)       # the whole load on the positions
    yf = _yfree(nel)
    d = np.linalg.solve(p.K[np.ix_(yf, yf)], Q[yf])               # small-deflection static solve
    sn = np.arange(1, nel + 1) * (L / nel)
    w = q * sn**2 * (6 * L**2 - 4 * L * sn + sn**2) / (24 * KB)
    ws = q * sn * (3 * L**2 - 3 * L * sn + sn**2) / (6 * KB)
    np.testing.assert_allclose(d[0::2], w, rtol=rtol)
    np.testing.assert_allclose(d[1::2], ws, rtol=rtol)
    assert d[-2] == pytest.approx(q * L**4 / (8 * KB), rel=rtol)  # tip: q L^4 / (8 E I)


def test_cantilever_frequencies():
    p = _plate()
    w2 = eigh(p.K[np.ix_(YF, YF)], p.M[np.ix_(YF, YF)], eigvals_only=True, subset_by_index=[0, 2])
    scale = math.sqrt(KB / (RHO * L**4))
    brackets = ((1.5, 2.5), (4.0, 5.0), (7.0, 8.5))
    for k, (a, b) in enumerate(brackets):
        x = brentq(lambda z: 1.0 + math.cos(z) * math.cosh(z), a, b)
        exact = x * x * scale
        # conforming elements bound each frequency from above (Rayleigh-Ritz); the gap grows
        # as (k h)^4: 1e-6 for the third mode at 40 elements
        assert exact * (1 - 1e-12) <= math.sqrt(w2[k]) <= exact * (1 + 5e-6)


def test_uniform_stretch_force():
    p = _plate()
    eps = 0.01
    for th in (0.0, 0.7):
        R = np.array([math.cos(th), math.sin(th)])
        e = np.zeros(p.ndof)
        for i in range(NEL + 1):
            e[4 * i:4 * i + 2] = (1 + eps) * i * (L / NEL) * R
            e[4 * i + 2:4 * i + 4] = (1 + eps) * R
        f = p.stretch_force(e)
        T = KS * eps * (1 + eps)                                    # K_S (|X_s| - 1) |X_s|
        expect = np.zeros(p.ndof)
        expect[0:2] = -T * R
        expect[-4:-2] = T * R
        # (the strain |X_s| - 1 comes from slopes summed with shape-function derivatives of
        # size 1/l, so it rounds to ~eps/l; the force carries K_S and another 1/l)
        l = L / NEL
        np.testing.assert_allclose(f, expect, atol=64 * np.finfo(float).eps * KS / l**2 * l)


def test_newmark_phase_on_the_first_mode():
    # bending only: the step (20 per period of the first mode) is far beyond the explicit
    # stretching part's stability limit, which this pin is not about
    p = _plate(k_s=0.0)
    w2, V = eigh(p.K[np.ix_(YF, YF)], p.M[np.ix_(YF, YF)], subset_by_index=[0, 0])
    w, phi = math.sqrt(w2[0]), V[:, 0] / np.abs(V[:, 0]).max()
    amp = 1e-3
    e = p.e.copy()
    e[YF] += amp * phi
    p.set_state(e, np.zeros(p.ndof), 0.0)
    dt = 0.05 / w * 2 * math.pi   # 20 steps per period
    wt = 2.0 * math.atan(0.5 * w * dt) / dt
    tip = []
    for n in range(1, 61):
        p.step(np.zeros((2, 64)), dt)
        tip.append(p.e[YF][-2] / (amp * phi[-2]))
    # (the computed mode carries rounding-level components of the stiff modes, about
    # eps lambda_max / lambda_1, which the rule keeps undamped: 1e-6 at the tip; the phase
    # distortion tested is 0.15 rad after 60 steps)
    np.testing.assert_allclose(tip, np.cos(wt * dt * np.arange(1, 61)), atol=2e-6)
    assert abs(wt - w) > 1e-3 * w    # the distortion is visible at this step


def test_constant_velocity_transport_stays_straight():
    U = np.array([0.3, -0.2])
    d0 = np.array([math.cos(0.4), -math.sin(0.4)])

    def clamp(t):
        z = np.zeros(2)
        return U * t, d0, U, z, z, z

    p = _plate(clamp=clamp)
    for _ in range(25):
        p.step(np.zeros((2, 64)), 0.01)
    X, V = p.markers()
    s = p.s_mark
    np.testing.assert_allclose(X, (U * p.t)[:, None] + d0[:, None] * s, atol=1e-13)
    np.testing.assert_allclose(V, np.broadcast_to(U[:, None], V.shape), atol=1e-13)


def test_straight_plate_markers_equal_the_rigid_plate():
    case = W.config5(n=128, L=8.0, nmark=64)
    pl = case.extra["plate"]
    for t0 in (0.0, 13.7):
        p = Plate(1.0, NEL, RHO, KS, KB, pl["s"], case.markers["dV"], flapping_clamp(pl), t0=t0)
        X, U = p.markers()
        Xr, Ur = W.plate_kinematics(case, t0)
        np.testing.assert_allclose(X, Xr, atol=1e-14)
        np.testing.assert_allclose(U, Ur, atol=1e-14)


def test_flapping_clamp_derivatives():
    case = W.config5(n=128, L=8.0, nmark=64)
    c = flapping_clamp(case.extra["plate"])
    for t in (0.0, 5.1, 40.3):
        h = 1e-3
        for k in range(2):   # position, slope
            np.testing.assert_allclose(c(t)[2 + k], (c(t + h)[k] - c(t - h)[k]) / (2 * h), atol=1e-8)
            np.testing.assert_allclose(c(t)[4 + k], (c(t + h)[k] - 2 * c(t)[k] + c(t - h)[k]) / h**2, atol=1e-6)


def test_accelerating_clamp_equals_a_body_load():
    # a clamp accelerating uniformly by g deforms the plate as a clamp at rest under the load
    # -rho_s g per unit length (the rule integrates the quadratic rigid motion exactly)
    g = np.array([0.02, -0.05])
    s, dv = _gauss_markers()

    def accel(t):
        z = np.zeros(2)
        return 0.5 * g * t * t, np.array([1.0, 0.0]), g * t, z, g, z

    pa = _plate(clamp=accel, s_mark=s, dv=dv)
    pr = _plate(s_mark=s, dv=dv)
    F = np.zeros((2, len(s)))
    Fl = np.broadcast_to((-RHO * g)[:, None], F.shape)
    pr.set_state(pr.e, pr.v, 0.0)
    pr.a[4:] = np.linalg.solve(pr.M[4:, 4:], pr.load(Fl)[4:])   # the loaded plate's start
    for _ in range(40):
        pa.step(F, 0.002)
        pr.step(Fl, 0.002)
    Xa, _ = pa.markers()
    Xr, _ = pr.markers()
    np.testing.assert_allclose(Xa - (0.5 * g * pa.t**2)[:, None], Xr, atol=1e-13)
    assert np.abs(Xr[1] - 0.0).max() > 1e-6      # it has bent
