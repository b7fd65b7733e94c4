"""Pins of the oracle's fifth-order reconstruction (WENO5-JS and TENO5, the schemes Sec. 2
names) and of the convective flux difference built on it.

* linear-weight limit: on data where the smoothness indicators coincide (WENO) or every
  sub-stencil is kept (TENO) the face value is the upwind-biased fifth-order value
  (2a - 13b + 47c + 27d - 3e)/60;
* a TENO example worked by hand (golden file);
* fifth-order convergence of (f_{i+1/2} - f_{i-1/2})/h to f' on smooth data;
* the convective term of the full right-hand side converges at fifth order to -dF/dx of an
  analytic state.
"""
import math
import os

import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def upwind5(v):
    a, b, c, d, e = v
    return (2 * a - 13 * b + 47 * c + 27 * d - 3 * e) / 60.0


def test_linear_weight_limit_weno(oracle_mod):
    rng = np.random.default_rng(0)
    for _ in range(50):
        s, o = rng.normal(), rng.normal()
        v = o + s * np.arange(5.0)              # linear data: all beta_k equal
        got = oracle_mod.recon5(v, "weno5js")
        assert got == pytest.approx(upwind5(v), rel=1e-13, abs=1e-13)


def test_linear_weight_limit_teno(oracle_mod):
    rng = np.random.default_rng(1)
    x = np.arange(-2, 3) * 0.01
    for _ in range(50):
        c = rng.normal(size=4)
        v = c[0] + c[1] * np.sin(x + c[2]) + 0.1 * c[3] * x ** 2   # smooth, well resolved
        assert oracle_mod.teno_flags(v) == 7
        assert oracle_mod.recon5(v, "teno5") == pytest.approx(upwind5(v), rel=1e-13, abs=1e-15)


def test_teno_worked_example(oracle_mod):
    rows = np.loadtxt(os.path.join(GOLDEN, "teno_worked_example.txt"))
    for row in rows:
        v, flags, val = row[:5], int(row[5]), row[6]
        assert oracle_mod.teno_flags(v) == flags
        assert oracle_mod.recon5(v, "teno5") == pytest.approx(val, rel=1e-15, abs=0)


def test_weno_step_is_essentially_non_oscillatory(oracle_mod):
    # across a jump the face value stays within the data range
    for v in ([0, 0, 0, 1, 1], [1, 1, 0, 0, 0], [0, 0, 1, 1, 1]):
        f = oracle_mod.recon5(v, "weno5js")
        assert -1e-3 < f < 1 + 1e-3


def _fd_derivative_error(oracle_mod, scheme, n, func, dfunc, x0=0.0, x1=1.0):
    h = (x1 - x0) / n
    x = x0 + (np.arange(-3, n + 3) + 0.5) * h     # exact ghost values
    f = func(x)
    faces = np.array([oracle_mod.recon5(f[i - 2:i + 3], scheme) for i in range(2, n + 4)])
    # faces[k] is the value at x_{k+2} + h/2 in the extended indexing; cell i (0-based
    # interior) uses faces (i+1) - (i)
    deriv = (faces[1:n + 1] - faces[0:n]) / h
    xi = x0 + (np.arange(n) + 0.5) * h
    return np.abs(deriv - dfunc(xi)).max()


@pytest.mark.parametrize("scheme", ["weno5js", "teno5"])
def test_fifth_order_on_exp(oracle_mod, scheme):
    errs = [_fd_derivative_error(oracle_mod, scheme, n, np.exp, np.exp) for n in (16, 32, 64, 128)]
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(slopes[1:]) > 4.7, (errs, slopes)


def test_teno_equals_upwind5_on_periodic_sine(oracle_mod):
    n = 64
    x = (np.arange(n) + 0.5) / n
    f = np.sin(2 * np.pi * x)
    fe = np.concatenate([f[-3:], f, f[:3]])
    for i in range(3, n + 3):
        v = fe[i - 2:i + 3]
        assert oracle_mod.recon5(v, "teno5") == pytest.approx(upwind5(v), rel=0, abs=1e-15)


def _analytic_case(n, scheme):
    # 1D-in-x periodic state: rho = 1 + 0.2 sin, u = 0.3 + 0.1 cos, p = 1/gamma (1 + 0.1 sin 2)
    return W.periodic_box(dim=2, n=n, scheme=scheme, terms=W.TERM["conv_x"])


def _analytic_fields(x, g):
    k = 2 * np.pi
    rho = 1 + 0.2 * np.sin(k * x)
    u = 0.3 + 0.1 * np.cos(k * x)
    p = (1 / g) * (1 + 0.1 * np.sin(2 * k * x))
    drho = 0.2 * k * np.cos(k * x)
    du = -0.1 * k * np.sin(k * x)
    dp = (1 / g) * 0.2 * k * np.cos(2 * k * x)
    E = p / (g - 1) + 0.5 * rho * u * u
    dE = dp / (g - 1) + 0.5 * drho * u * u + rho * u * du
    # x-fluxes and their derivatives
    dF = [drho * u + rho * du,
          drho * u * u + 2 * rho * u * du + dp,
          0 * x,
          (dE + dp) * u + (E + p) * du]
    return rho, u, p, dF


@pytest.mark.parametrize("scheme", ["weno5js", "teno5"])
def test_convective_term_fifth_order(oracle_mod, scheme):
    errs = []
    for n in (64, 128, 256):
        case = _analytic_case(n, scheme)
        xs = W.centres(case)
        rho, u, p, dF = _analytic_fields(xs[0], case.gamma)
        Q = W.conserved(case, rho, [u, 0 * u], p)
        L = oracle_mod.Oracle(case).rhs(Q)
        errs.append(max(np.abs(L[m] + dF[m]).max() for m in range(4)))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert slopes[-1] > 4.7, (errs, slopes)


def test_weno_js_rational_examples(oracle_mod):
    rows = np.loadtxt(os.path.join(GOLDEN, "weno_js_examples.txt"))
    for row in rows:
        got = oracle_mod.recon5(row[:5], "weno5js")
        assert got == pytest.approx(row[5], rel=1e-13)
