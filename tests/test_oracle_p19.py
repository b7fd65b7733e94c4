"""Pin P19: the paper's one qualitative comparison of its two schemes (Sec. 3, scattering by a
stationary sphere): with the periodic Gaussian pressure source, TENO5's pressure peaks along
the +x axis beyond the source are at least WENO5-JS's (TENO5 is the less dissipative).

A miniature of that set-up: the sphere of radius R = 0.5 on [-3, 3]^3 at 64^3 (about five
cells per wavelength of the source), the source at 2R with the paper's A, B and omega, the
gas at rest at the start, three source periods; the envelope (largest |Delta p| over the run)
at probes on +x between x = 1.3 and 1.9 (x / R = 2.6 .. 3.8, past the source, inside the
sponge).  Only the oracle computes; about a minute of host time.
"""
import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W


@pytest.mark.slow
def test_teno5_peaks_at_least_weno5js_along_x(oracle_mod):
    env = {}
    for scheme in ("teno5", "weno5js"):
        case = W.config3_source(n=64, scheme=scheme, nmark=2000, L=6.0)
        xs = np.arange(1.3, 1.9001, case.h / 2)
        o = oracle_mod.Oracle(case.with_(probes=np.stack([xs, 0 * xs, 0 * xs])))
        Q = W.uniform_state(case)
        steps = int(round(1.5 / case.dt))                  # three periods of 2 pi / omega = 0.5
        peak = np.zeros(xs.size)
        for _ in range(steps):
            o.rk3_step(Q, case.dt)
            peak = np.maximum(peak, np.abs(o.probe_dp(Q)))
        env[scheme] = peak
    t, w = env["teno5"], env["weno5js"]
    assert w.max() > 1e-5                                  # the waves have reached the probes
    assert (t >= w).all(), np.nonzero(t < w)
    assert t.max() > 1.005 * w.max()
