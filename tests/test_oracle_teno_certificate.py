"""The all-kept certificate the 3D face passes use as a wave-wide shortcut, against the
oracle's TENO5 decision (Sec. 2's cut-off of chi_k = gamma_k / sum gamma at C_T,
gamma_k = (1 + tau5 / (beta_k + eps))^6): whenever tau5 <= T (beta_min + eps) with
T = (3 C_T)^(-1/6) * 0.99 - 1, the oracle keeps every sub-stencil, over stencils of every kind
(smooth, noisy, flat to rounding, exactly flat, steps, scales from 1e-150 to 1e150) and several
cut-offs; and the bound lies within 2% below the exact one of the derivation, which no
stencil the oracle cuts falls under."""
import numpy as np
import pytest

EPS = 1e-40


def _bound(ct):
    return (3.0 * ct) ** (-1.0 / 6.0) * (1.0 - 1e-2) - 1.0 if ct < 1.0 / 3.0 else -1.0


def _betas(v):
    a, b, c, d, e = v.T
    b0 = 13.0 / 12.0 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2
    b1 = 13.0 / 12.0 * (b - 2 * c + d) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * (c - 2 * d + e) ** 2 + 0.25 * (3 * c - 4 * d + e) ** 2
    return b0, b1, b2


def _stencils(rng, n):
    x = np.arange(5.0) - 2.0
    kinds = [
        rng.normal(size=(n, 1)) + rng.normal(size=(n, 1)) * x + 0.1 * rng.normal(size=(n, 1)) * x**2,  # smooth
        rng.normal(size=(n, 5)),                                                                        # noise
        1.0 + 1e-15 * rng.normal(size=(n, 5)),                                                          # flat to rounding
        np.repeat(rng.uniform(0.1, 3.0, size=(n, 1)), 5, axis=1),                                       # exactly flat
        np.where(x > rng.integers(-2, 3, size=(n, 1)) - 0.5, 1.0, 0.0) + 1e-3 * rng.normal(size=(n, 5)),  # steps
    ]
    v = np.concatenate(kinds)
    scale = 10.0 ** rng.uniform(-150, 150, size=(v.shape[0], 1))
    return np.concatenate([v, v * scale])


@pytest.mark.parametrize("ct", [1e-6, 1e-5, 1e-3, 0.2, 0.34])
def test_certificate_implies_every_sub_stencil_kept(oracle_mod, ct):
    rng = np.random.default_rng(int(ct * 1e7) + 7)
    V = _stencils(rng, 4000)
    b0, b1, b2 = _betas(V)
    cert = np.abs(b0 - b2) <= _bound(ct) * (np.minimum(np.minimum(b0, b1), b2) + EPS)
    flags = oracle_mod.teno_flags_n(np.ascontiguousarray(V), teno_ct=ct, teno_eps=EPS)
    assert (flags[cert] == 7).all(), V[cert & (flags != 7)][:3]
    if ct < 1.0 / 3.0:
        assert cert.sum() > 0.2 * len(V)      # it holds on a good share of these stencils
    else:
        assert cert.sum() == 0                # no certificate for C_T >= 1/3


def test_bound_is_close_to_the_cut_off(oracle_mod):
    # the bound sits within 2% below the exact limit (3 C_T)^(-1/6) - 1 of tau5 / (beta_min +
    # eps), under which no sub-stencil can be cut; a family of stencils (a ramp with a kink of
    # growing size) crosses from kept to cut above that limit
    ct = 1e-6
    exact = (3.0 * ct) ** (-1.0 / 6.0) - 1.0
    assert 0.98 * (exact + 1.0) <= _bound(ct) + 1.0 <= exact + 1.0
    # a linear ramp plus a kink: vary the kink until the oracle's decision changes
    x = np.arange(5.0) - 2.0
    kept_ratio, cut_ratio = [], []
    for k in np.geomspace(1e-4, 1e4, 400):
        v = x + k * np.maximum(x, 0.0) ** 2
        b0, b1, b2 = _betas(v[None, :])
        r = float(np.abs(b0 - b2)[0] / (min(b0[0], b1[0], b2[0]) + EPS))
        f = oracle_mod.teno_flags_n(np.ascontiguousarray(v[None, :]), teno_ct=ct, teno_eps=EPS)[0]
        (kept_ratio if f == 7 else cut_ratio).append(r)
    assert kept_ratio and cut_ratio
    # every stencil the oracle cuts lies above the exact limit (the derivation); TENO5's own
    # structure (tau5 = |beta_0 - beta_2| also raises the cut sub-stencil's gamma) puts this
    # family's first cut at ~2.7 times it
    assert min(cut_ratio) > exact
