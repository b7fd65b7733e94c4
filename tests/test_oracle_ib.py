"""Pins of the oracle's immersed-boundary operators (Sec. 2, Eqs. (8)-(11)).

The four-point function is checked against values worked by hand from Eq. (11) and against
Peskin's moment conditions; interpolation and spreading against exactness on affine fields,
conservation of total force and torque, and their adjointness.
"""
import os

import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_delta4_hand_values(oracle_mod):
    rows = np.loadtxt(os.path.join(GOLDEN, "delta4_values.txt"))
    for r, v in rows:
        assert oracle_mod.delta4(r) == pytest.approx(v, abs=2e-16)


def test_delta4_moments(oracle_mod):
    rng = np.random.default_rng(1)
    for r in rng.uniform(-3, 3, size=200):
        js = np.arange(np.floor(r) - 3, np.floor(r) + 4)
        phi = np.array([oracle_mod.delta4(r - j) for j in js])
        assert abs(phi.sum() - 1.0) < 1e-15                      # zeroth moment
        assert abs(((r - js) * phi).sum()) < 1e-15                # first moment
        assert abs((phi ** 2).sum() - 0.375) < 1e-15              # sum of squares 3/8
        even = (js % 2 == 0)
        assert abs(phi[even].sum() - 0.5) < 1e-15                 # even/odd split
        assert abs(phi[~even].sum() - 0.5) < 1e-15
        assert (phi >= 0).all()


def _ib_case(dim, n=24, nmark=40, seed=0):
    case = W.periodic_box(dim=dim, n=n, L=1.0)
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.25, 0.75, size=(dim, nmark))
    dV = rng.uniform(0.5, 1.5, size=nmark) * case.h ** (dim - 1)
    return case.with_(markers={"X": X, "dV": dV, "U": None, "motion": "static", "omega": 0.0})


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_exact_on_affine(oracle_mod, dim):
    case = _ib_case(dim)
    o = oracle_mod.Oracle(case)
    xs = W.centres(case)
    coef = np.array([0.3, -1.7, 2.2, 0.9])
    field = np.stack([coef[0] + sum(coef[1 + d] * xs[d] for d in range(dim)),
                      -1.0 + 0.5 * xs[0]])
    got = o.ib_interp(field)
    X = case.markers["X"]
    want0 = coef[0] + sum(coef[1 + d] * X[d] for d in range(dim))
    want1 = -1.0 + 0.5 * X[0]
    np.testing.assert_allclose(got[0], want0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(got[1], want1, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_spread_force_and_torque(oracle_mod, dim):
    case = _ib_case(dim, seed=3)
    o = oracle_mod.Oracle(case)
    rng = np.random.default_rng(5)
    F = rng.normal(size=(dim, o.nm))
    f = np.zeros((dim,) + case.shape)
    o.ib_spread(F, f)
    hd = case.h ** dim
    dV = case.markers["dV"]
    X = case.markers["X"]
    total = np.array([f[a].sum() * hd for a in range(dim)])
    np.testing.assert_allclose(total, -(F * dV).sum(axis=1), rtol=1e-13, atol=1e-15)
    xs = W.centres(case)
    # torque about the origin, z component
    tz = (xs[0] * f[1] - xs[1] * f[0]).sum() * hd
    tz_m = -((X[0] * F[1] - X[1] * F[0]) * dV).sum()
    assert tz == pytest.approx(tz_m, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_spread_adjoint(oracle_mod, dim):
    case = _ib_case(dim, seed=7)
    o = oracle_mod.Oracle(case)
    rng = np.random.default_rng(9)
    u = rng.normal(size=(dim,) + case.shape)
    F = rng.normal(size=(dim, o.nm))
    Iu = o.ib_interp(u)
    f = np.zeros_like(u)
    o.ib_spread(F, f)
    lhs = (Iu * F * case.markers["dV"]).sum()
    rhs = -(u * f).sum() * case.h ** dim
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_marker_outside_grid_rejected(oracle_mod):
    case = W.periodic_box(dim=2, n=16)
    o = oracle_mod.Oracle(case)
    X = np.array([[0.01], [0.5]])   # support would reach cell -2
    with pytest.raises(ValueError):
        o.set_markers(X, np.ones(1))


def test_spread_accumulates_scale(oracle_mod):
    case = _ib_case(2, seed=11)
    o = oracle_mod.Oracle(case)
    F = np.ones((2, o.nm))
    f1 = np.zeros((2,) + case.shape)
    o.ib_spread(F, f1, 1.0)
    f2 = np.full((2,) + case.shape, 3.0)
    o.ib_spread(F, f2, -2.0)
    np.testing.assert_allclose(f2, 3.0 - 2.0 * f1, rtol=1e-15, atol=1e-15)


def _uniform_flow_case(u0, omega=0.3, alpha=7.0, beta=2.5, terms=W.TERM["ib"]):
    case = W.periodic_box(dim=2, n=32, terms=terms, prim_inf=(1.2, u0[0], u0[1], 0.0, 0.8))
    X, dV = W.circle_markers(16, 0.2, (0.0, 0.0))
    X = X + 0.5
    return case.with_(ib_alpha=alpha, ib_beta=beta,
                      markers={"X": X, "dV": dV, "U": None, "motion": "rotating", "omega": omega})


def test_penalty_force_law(oracle_mod):
    """Eq. (7): F = alpha xi + beta (U_ib - U); rotating markers move anticlockwise,
    U = omega (-(y - 0), x - 0) about the origin."""
    u0 = (0.13, -0.07)
    case = _uniform_flow_case(u0)
    o = oracle_mod.Oracle(case)
    X = case.markers["X"]
    U = 0.3 * np.stack([-X[1], X[0]])
    xi = np.random.default_rng(3).normal(size=(2, o.nm))
    o.set_state(xi, 0.0, 0)
    o.rhs(W.uniform_state(case))
    F = o.marker_force()
    # U_ib of a uniform field is exactly the field value (zeroth moment)
    want = 7.0 * xi + 2.5 * (np.array(u0)[:, None] - U)
    np.testing.assert_allclose(F, want, rtol=1e-13, atol=1e-14)


def test_ib_energy_source_is_force_work(oracle_mod):
    u0 = (0.11, 0.04)
    case = _uniform_flow_case(u0)
    o = oracle_mod.Oracle(case)
    L = o.rhs(W.uniform_state(case))
    assert np.all(L[0] == 0.0)
    np.testing.assert_allclose(L[3], L[1] * u0[0] + L[2] * u0[1], rtol=1e-13, atol=1e-18)
    assert np.abs(L[1]).max() > 0


def test_penalty_integral_advances_with_rk3(oracle_mod):
    """With alpha = beta = 0 the fluid is untouched, so U_ib - U is constant over the step
    and the SSP-RK3 stages must integrate it exactly: xi(dt) = xi(0) + dt (u0 - U)."""
    u0 = (0.09, 0.02)
    case = _uniform_flow_case(u0, omega=0.4, alpha=0.0, beta=0.0)
    o = oracle_mod.Oracle(case)
    xi0 = np.random.default_rng(4).normal(size=(2, o.nm))
    o.set_state(xi0, 0.0, 0)
    Q = W.uniform_state(case)
    dt = 0.05
    o.rk3_step(Q, dt)
    xi, t, step = o.get_state()
    X = case.markers["X"]
    U = 0.4 * np.stack([-X[1], X[0]])
    np.testing.assert_allclose(xi, xi0 + dt * (np.array(u0)[:, None] - U), rtol=1e-13, atol=1e-15)
    assert t == dt and step == 1
    # anticlockwise: the marker with the largest x moves in +y
    k = int(np.argmax(X[0]))
    assert U[1, k] > 0


def test_sponge_profile_hand_values(oracle_mod):
    rows = np.loadtxt(os.path.join(GOLDEN, "sponge_profile.txt"))
    case = W.periodic_box(dim=2, n=8, terms=W.TERM["sponge"])
    case = case.with_(sponge_width=((0.25, 0.0), (0.0, 0.0), (0.0, 0.0)), sponge_sigma=8.0)
    Q = W.uniform_state(case)
    Q[0] += 1e-3
    L = oracle_mod.Oracle(case).rhs(Q)
    for i, sg in rows:
        np.testing.assert_allclose(L[0][:, int(i)], -sg * 1e-3, rtol=1e-12, atol=1e-18)
