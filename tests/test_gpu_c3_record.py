"""The 256^3 sphere-scattering case at full size against the oracle's record of it: the
configured 500 SSP-RK3 steps from the pulse in WENO5-JS (continuous weights: the run is
determined to rounding), 10^4 markers, sponge, on the GPU in the benchmark's launch
configuration, against tests/golden/c3_oracle_run_weno5js.npz (written by c3_oracle_run.py
with the oracle alone). Held to the parity tests' bounds: R20's 1e-12 (relative L2 per
component, scaled by its natural size) and the element-wise bound on 8192 sampled cells after
steps 100, 250 and 500; the probe pressure to 1e-12 of p_inf; the force and the norms of
Q - Q0 to 1e-10 relative.
"""
import os

import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

from test_gpu_parity_2d import ELEM_ULPS, TOL_ELEM, _say, _solver, natural_scale

pytestmark = pytest.mark.gpu
RECORD = os.path.join(os.path.dirname(__file__), "golden", "c3_oracle_run_weno5js.npz")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_sphere_full_size_run_to_rounding():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(RECORD):
        pytest.skip("the oracle record has not been written (tests/golden/c3_oracle_run.py)")
    rec = np.load(RECORD)
    assert str(rec["scheme"]) == "weno5js"
    steps, every, norm_every = int(rec["steps"]), int(rec["every"]), int(rec["norm_every"])
    case = W.config3(n=256, scheme="weno5js")
    assert abs(float(rec["dt"]) - case.dt) == 0.0
    s = _solver(case)
    Q0 = W.config3_state(case)
    Q = torch.from_numpy(Q0.copy()).cuda()
    Q0g = torch.from_numpy(Q0).cuda()
    cells = torch.from_numpy(rec["cells"]).cuda()
    snap_steps = [int(x) for x in rec["snap_steps"]]
    dp, force, norms, dnorms, snaps = [], [], [], [], {}
    _say(f"c3 record: {steps} steps on the GPU")
    for k in range(steps // every):
        s.rk3_steps(Q, case.dt, every) if k == 0 else s.rk3_steps_resume(Q, case.dt, every)
        dp.append(s.probe_dp(Q).cpu().numpy())
        force.append((s.marker_force() * case.markers["dV"]).sum(axis=1))
        n = (k + 1) * every
        if n % norm_every == 0:
            norms.append([float(torch.linalg.norm(Q[c])) for c in range(case.nq)])
            dnorms.append([float(torch.linalg.norm(Q[c] - Q0g[c])) for c in range(case.nq)])
        if n in snap_steps:
            snaps[n] = Q.reshape(case.nq, -1)[:, cells].cpu().numpy()
    s.sync()
    dp, force = np.array(dp), np.array(force)
    p_inf = case.prim_inf[4]
    d = np.abs(dp - rec["dp"]).max()
    _say(f"  probes: max|d dp| {d:.2e} of signal {np.abs(rec['dp']).max():.2e}; force rel "
         f"{_rel(force, rec['force']):.2e}; |Q - Q0| norms rel {_rel(np.array(dnorms), rec['dnorms']):.2e}")
    assert np.abs(rec["dp"]).max() > 1e-6 * p_inf          # the pulse has reached the probes
    assert d <= 1e-12 * p_inf
    assert _rel(force, rec["force"]) <= 1e-10
    assert _rel(np.array(dnorms), rec["dnorms"]) <= 1e-10
    assert _rel(np.array(norms), rec["norms"]) <= 1e-12
    Q0s = Q0.reshape(case.nq, -1)[:, rec["cells"]]
    scale = natural_scale(case)
    for i, n in enumerate(snap_steps):
        g, o = snaps[n], rec["snaps"][i]
        for c in range(case.nq):
            rel = np.linalg.norm(g[c] - o[c]) / max(np.linalg.norm(o[c]), scale[c] * np.sqrt(o[c].size))
            dm, dev = np.abs(g[c] - o[c]).max(), np.abs(o[c] - Q0s[c]).max()
            _say(f"  step {n} component {c}: rel L2 {rel:.3e}, max|dQ| {dm:.3e} of change {dev:.3e}")
            assert rel <= 1e-12, (n, c, rel)
            assert dm <= TOL_ELEM * dev + ELEM_ULPS * np.finfo(float).eps * scale[c], (n, c, dm, dev)
