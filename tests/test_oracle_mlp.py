"""Pins of the learned-weight references: face features and labels (oracle/ora.c) and the
FP64 MLP with its gradient (oracle/mlp.py)."""
import math

import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W


@pytest.fixture(scope="module")
def mlp():
    from oracle import mlp as M

    return M


def test_bf16_rounding_known_values(mlp):
    # 1 + 2^-8 is the midpoint between 1 and 1 + 2^-7: ties go to the even mantissa (1.0);
    # 1 + 3 * 2^-8 ties between 1 + 2^-7 and 1 + 2^-6 and goes to 1 + 2^-6.
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 3.0e-30])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, np.float32(3.0e-30)])
    got = mlp.bf16(vals)
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == want[2] and got[3] == want[3] and got[4] == -2.5
    assert abs(got[5] - 3e-30) / 3e-30 < 2 ** -8


def test_zero_network_loss_is_ln2(mlp):
    theta = np.zeros(mlp.NPARAM)
    X = np.random.default_rng(0).uniform(-1, 1, size=(50, 15))
    Y = np.random.default_rng(1).integers(0, 2, size=(50, 3))
    loss, g = mlp.loss_and_grad(theta, X, Y)
    assert loss == pytest.approx(math.log(2.0), rel=1e-15)


def test_gradient_against_finite_differences(mlp):
    rng = np.random.default_rng(2)
    theta = mlp.init_params(3) + 0.05 * rng.normal(size=mlp.NPARAM)
    X = rng.uniform(-1, 1, size=(40, 15))
    Y = rng.integers(0, 2, size=(40, 3))
    _, g = mlp.loss_and_grad(theta, X, Y)
    idx = rng.choice(mlp.NPARAM, size=60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, X, Y)[0] - mlp.loss_and_grad(tm, X, Y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_moves_by_lr(mlp):
    # with bias correction the first Adam step is -lr * sign(g) (up to eps)
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = mlp.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 0.01)
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-4)


def test_training_fits_a_separable_rule(mlp):
    # a tiny problem the network must learn: bit k = feature k > 0
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, size=(512, 15))
    Y = (X[:, :3] > 0).astype(float)
    theta = mlp.init_params(5)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss_and_grad(theta, X, Y)[0]
    for t in range(1, 301):
        _, g = mlp.loss_and_grad(theta, X, Y)
        theta, m, v = mlp.adam(theta, m, v, g, t, 0.01)
    l1 = mlp.loss_and_grad(theta, X, Y)[0]
    bits, _ = mlp.keep_flags(mlp.forward(theta, X)[0])
    acc = np.mean(bits == (Y[:, 0] + 2 * Y[:, 1] + 4 * Y[:, 2]))
    assert l1 < 0.3 * l0 and acc > 0.9


def _row_case(n=24):
    return W.periodic_box(dim=2, n=n, scheme="teno5").with_(
        bc=(("extrap", "extrap"), ("periodic", "periodic"), ("periodic", "periodic")))


def test_features_of_linear_and_constant_stencils(oracle_mod):
    case = _row_case()
    xs = W.centres(case)
    h = case.h
    rho = 1.0 + 0.01 * xs[0]
    Q = W.conserved(case, rho, [0.1 + 0 * rho, 0 * rho], np.full(case.shape, 0.7))
    o = oracle_mod.Oracle(case)
    # deviations 0.01 h (k - 2) over the largest one 0.02 h plus the floor 1e-8 rho_inf
    r = 0.02 * h / (0.02 * h + 1e-8)
    f0 = o.face_features(Q, 0, (10, 5), 0)
    np.testing.assert_allclose(f0[:5], [-r, -r / 2, 0, r / 2, r], rtol=1e-9, atol=0)
    assert 0.99998 < r < 0.99999
    np.testing.assert_allclose(f0[5:], 0.0, atol=0)          # u and p constant
    f1 = o.face_features(Q, 0, (10, 5), 1)                     # mirrored: cells 13..9
    np.testing.assert_allclose(f1[:5], [r, r / 2, 0, -r / 2, -r], rtol=1e-9, atol=0)
    # normal velocity is negated on the mirrored side (c_inf = 1 here)
    Q2 = W.conserved(case, 1.0 + 0 * rho, [0.1 + 0.01 * xs[0], 0 * rho], np.full(case.shape, 0.7))
    g0 = o.face_features(Q2, 0, (10, 5), 0)
    g1 = o.face_features(Q2, 0, (10, 5), 1)
    np.testing.assert_allclose(g0[5:10], [-r, -r / 2, 0, r / 2, r], rtol=1e-9)
    np.testing.assert_allclose(g1[5:10], [-r, -r / 2, 0, r / 2, r], rtol=1e-9)


def test_features_of_rounding_level_variation_vanish(oracle_mod):
    # p varying by 1e-15 (rounding level): the floor 1e-8 rho c^2 = 1e-8 maps it to ~1e-7
    case = _row_case()
    xs = W.centres(case)
    p = 0.7 + 1e-15 * np.sign(np.sin(7.0 * xs[0]))
    Q = W.conserved(case, np.ones(case.shape), [0 * p + 0.1, 0 * p], p)
    f = oracle_mod.Oracle(case).face_features(Q, 0, (10, 5), 0)
    assert np.abs(f[10:]).max() < 1e-6


def test_significance(oracle_mod):
    case = _row_case()
    xs = W.centres(case)
    o = oracle_mod.Oracle(case)
    const = W.uniform_state(case)
    assert not o.face_significant(const, 0, (10, 5), 0)
    for var, amp, want in (("rho", 0.9e-8, False), ("rho", 1.1e-8, True), ("v", 1.1e-8, True),
                           ("v", 0.9e-8, False), ("p", 1.1e-8, True)):
        # a jump of amp (natural scales are 1 here) between cells 11 and 12
        jump = amp * (np.arange(case.n[0])[None, :] >= 12)
        rho = 1.0 + (jump if var == "rho" else 0)
        v = 0.0 + (jump if var == "v" else 0)
        p = 1.0 / 1.4 + (jump if var == "p" else 0)
        Q = W.conserved(case, rho * np.ones(case.shape), [0.0 * rho + 0.1, v * np.ones(case.shape)],
                        p * np.ones(case.shape))
        assert o.face_significant(Q, 0, (10, 5), 0) == want, (var, amp)
        assert not o.face_significant(Q, 0, (6, 5), 0)          # cells 4..8: no jump


def test_labels_smooth_and_step(oracle_mod):
    case = _row_case()
    xs = W.centres(case)
    o = oracle_mod.Oracle(case)
    # linear data: all smoothness indicators equal, tau5 = 0, every sub-stencil kept
    smooth = W.conserved(case, 1.0 + 0.01 * xs[0], [0.05 + 0.02 * xs[0], 0 * xs[0]],
                         np.full(case.shape, 0.7))
    assert o.face_label(smooth, 0, (10, 5), 0, 1.2) == 7
    assert o.face_label(smooth, 0, (10, 5), 1, 1.2) == 7
    # density jump between cells 11 and 12: for the face 10|11 side 0 uses cells 8..12, so
    # sub-stencil 2 = (10, 11, 12) contains the jump and is cut; S0 and S1 are smooth.
    rho = np.where(np.arange(case.n[0])[None, :] >= 12, 1.5, 1.0) * np.ones(case.shape)
    step = W.conserved(case, rho, [0 * rho, 0 * rho], np.full(case.shape, 0.7))
    assert o.face_label(step, 0, (10, 5), 0, 1.2) == 3
    # side 1 uses cells 13, 12, 11, 10, 9: S0 = (13, 12, 11) and S1 = (12, 11, 10) contain the
    # jump, only S2 = (11, 10, 9) is kept; the momentum and energy fluxes are constant here
    # and count as keeping everything
    assert o.face_label(step, 0, (10, 5), 1, 1.2) == 4
