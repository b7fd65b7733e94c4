"""The benchmarked run itself against the oracle: the 2048^2 rotating-cylinder case (TENO5,
512 markers, inflow with the seeded perturbation, sponge), 4000 SSP-RK3 steps from the
uniform start on the GPU in the benchmark's launch configuration, against the CPU oracle's
record of the same run (tests/golden/c2_oracle_run.npz, written by c2_oracle_run.py with the
oracle alone). Compared quantities: the acoustic pressure on the configured radius-50 ring
and on a radius-10 ring every 10 steps, the total penalty force every 10 steps, per-component
norms every 100 steps, and 8192 sampled cells after steps 500, 1000, 2000, 3000 and 4000.

This run is not determined beyond rounding. From the uniform start, TENO5's sharp cut-off
meets stencils whose chi_k lies within rounding of C_T. A tie on a stencil that varies
strongly (test_gpu_teno_ties: relative spreads up to 0.35 on this set-up) changes the face
value by a good part of that variation, and the start-up transient carries the change on.

Two correct FP64 implementations therefore part ways after a few tens of steps, and so does
either one from itself. Started from the same state moved by at most one ulp per value, the
oracle's run departs from its own record by 1.2e-6 (relative) in the y-momentum norm at step
40 and by 3.7e-7 at step 100; the two runs agree to 2e-9 at step 30.

So the test holds the library's distance from the oracle to the scale of that
indeterminacy. A second GPU run gets one ulp of seeded rounding noise added to every value
after every 10 steps, the size of the differences two implementations' roundings make. The
library's distance from the oracle must stay within ENVELOPE times its distance from that
noisy run. Measured ratios lie between 0.69 and 2.14 over probes, force, norms and every
sampled component, so the library is as far from the oracle as it is from itself.

It must also stay within 1% on both probe rings where they carry the start-up wave (measured
5.4e-4 at r = 50 over 4000 steps, 1.1e-3 at r = 10), within 1% in the force (2.5e-3) and the
norms of Q - Q0 (3.5e-4), and within 10% of the sampled state's change. The largest measured
gap is 6.3% of the density change in the near wake at step 2000, where the noisy run
differs by 6.0%.
"""
import os

import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

from test_gpu_parity_2d import _say, _solver

pytestmark = pytest.mark.gpu
RECORD = os.path.join(os.path.dirname(__file__), "golden", "c2_oracle_run.npz")
ENVELOPE = 4.0
PHYS = 1e-2
SNAP_PHYS = 0.1


@pytest.fixture(scope="module")
def runs():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(RECORD):
        pytest.skip("the oracle record has not been written (tests/golden/c2_oracle_run.py)")
    rec = np.load(RECORD)
    steps, every, norm_every = int(rec["steps"]), int(rec["every"]), int(rec["norm_every"])
    case = W.config2()
    assert abs(float(rec["dt"]) - case.dt) == 0.0 and int(rec["seed"]) == case.seed
    nprobe = case.probes.shape[1]
    rings = case.with_(probes=np.concatenate([case.probes, W.ring_probes(nprobe, 10.0)], axis=1))
    Q0 = W.config2_state(case)
    Q0g = torch.from_numpy(Q0).cuda()
    cells = torch.from_numpy(rec["cells"]).cuda()
    snap_steps = [int(x) for x in rec["snap_steps"]]
    out = {}
    for label, noisy in (("gpu", False), ("gpu_noisy", True)):
        s = _solver(rings)
        Q = Q0g.clone()
        gen = torch.Generator(device="cuda")
        gen.manual_seed(1905)
        up = torch.full_like(Q, float("inf"))
        dp, force, norms, dnorms, snaps = [], [], [], [], {}
        _say(f"c2 record: {steps} steps on the GPU ({label})")
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
            if noisy:
                # one ulp up or down at every value (seeded), in place
                sign = torch.randint(0, 2, Q.shape, device="cuda", generator=gen, dtype=torch.int8)
                Q.copy_(torch.nextafter(Q, torch.where(sign.bool(), up, -up)))
        s.sync()
        out[label] = {"dp": np.array(dp), "force": np.array(force), "norms": np.array(norms),
                      "dnorms": np.array(dnorms), "snaps": snaps}
        s.close()
    out.update(rec=rec, case=case, nprobe=nprobe, every=every, Q0=Q0)
    return out


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _check(rows, name, to_oracle, to_noisy, phys=None):
    ratio = to_oracle / to_noisy if to_noisy > 0 else np.inf
    _say(f"  {name}: library vs oracle {to_oracle:.3e}; library vs its noisy run {to_noisy:.3e} (ratio {ratio:.2f})")
    rows.append((name, to_oracle, to_noisy, phys))


def _assert_rows(rows):
    for name, to_oracle, to_noisy, phys in rows:
        assert to_noisy > 0.0, name
        assert to_oracle <= ENVELOPE * to_noisy, (name, to_oracle, to_noisy)
        if phys is not None:
            assert to_oracle <= phys, (name, to_oracle)


@pytest.mark.parametrize("upto", [2000, 4000])
def test_probe_pressure(runs, upto):
    """Delta p on both rings (the radius-10 ring through step 2000, as recorded)."""
    rec, npr, k = runs["rec"], runs["nprobe"], upto // runs["every"]
    g, z = runs["gpu"]["dp"][:k], runs["gpu_noisy"]["dp"][:k]
    o50 = rec["dp_r50"][:k]
    k10 = min(k, rec["dp_r10"].shape[0])
    o10 = rec["dp_r10"][:k10]
    p_inf = runs["case"].prim_inf[4]
    rows = []
    # the 1% bound where the ring carries the start-up wave (up to step 2000 the radius-50 ring
    # sees only its 1e-8 precursor, relative errors of which say nothing)
    _check(rows, f"r = 50 ring to step {upto} (signal up to {np.abs(o50).max():.2e})", _rel(g[:, :npr], o50),
           _rel(g[:, :npr], z[:, :npr]), PHYS if np.abs(o50).max() > 1e-4 * p_inf else None)
    _check(rows, f"r = 10 ring to step {min(upto, 2000)} (signal up to {np.abs(o10).max():.2e})",
           _rel(g[:k10, npr:], o10), _rel(g[:k10, npr:], z[:k10, npr:]), PHYS)
    _assert_rows(rows)
    if upto == 4000:
        # the start-up wave has crossed the configured ring
        assert np.abs(o50).max() > 1e-3 * p_inf


@pytest.mark.parametrize("upto", [2000, 4000])
def test_force_and_norms(runs, upto):
    rec = runs["rec"]
    k, m = upto // runs["every"], upto // int(rec["norm_every"])
    g, z = runs["gpu"], runs["gpu_noisy"]
    rows = []
    _check(rows, f"marker force to step {upto}", _rel(g["force"][:k], rec["force"][:k]),
           _rel(g["force"][:k], z["force"][:k]), PHYS)
    _check(rows, f"|Q - Q0| norms to step {upto}", _rel(g["dnorms"][:m], rec["dnorms"][:m]),
           _rel(g["dnorms"][:m], z["dnorms"][:m]), PHYS)
    _assert_rows(rows)
    assert _rel(g["norms"][:m], rec["norms"][:m]) <= 1e-6       # the norms of Q itself: ambient-dominated


def test_sampled_state(runs):
    rec, case = runs["rec"], runs["case"]
    Q0s = runs["Q0"].reshape(case.nq, -1)[:, rec["cells"]]
    rows = []
    for i, n in enumerate(int(x) for x in rec["snap_steps"]):
        g, z, o = runs["gpu"]["snaps"][n], runs["gpu_noisy"]["snaps"][n], rec["snaps"][i]
        for c in range(case.nq):
            # relative to the change since the start, per component
            _check(rows, f"step {n} component {c} (change up to {np.abs(o[c] - Q0s[c]).max():.2e})",
                   _rel(g[c] - Q0s[c], o[c] - Q0s[c]), _rel(g[c] - Q0s[c], z[c] - Q0s[c]), SNAP_PHYS)
    _assert_rows(rows)


RECORD_WENO = os.path.join(os.path.dirname(__file__), "golden", "c2_oracle_run_weno5js_200.npz")


def test_weno5js_companion_run_to_rounding():
    """The same 2048^2 set-up in WENO5-JS, whose continuous weights leave the run determined to
    rounding: 200 steps from the uniform start against the oracle's record of them
    (c2_oracle_run_weno5js_200.npz), held to the parity tests' bounds -- R20's 1e-12 (relative
    L2 per component, scaled by its natural size) and the element-wise bound on the sampled
    state after the last step, the probe pressure to 1e-12 of p_inf, force and norms to 1e-10
    relative."""
    import torch

    from test_gpu_parity_2d import ELEM_ULPS, TOL_ELEM, natural_scale

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(RECORD_WENO):
        pytest.skip("the WENO5-JS record has not been written (tests/golden/c2_oracle_run.py --scheme weno5js)")
    rec = np.load(RECORD_WENO)
    assert str(rec["scheme"]) == "weno5js"
    steps, every, norm_every = int(rec["steps"]), int(rec["every"]), int(rec["norm_every"])
    case = W.config2().with_(scheme="weno5js")
    assert abs(float(rec["dt"]) - case.dt) == 0.0
    nprobe = case.probes.shape[1]
    s = _solver(case.with_(probes=np.concatenate([case.probes, W.ring_probes(nprobe, 10.0)], axis=1)))
    Q0 = W.config2_state(case)
    Q = torch.from_numpy(Q0.copy()).cuda()
    dp, force, norms = [], [], []
    for k in range(steps // every):
        s.rk3_steps(Q, case.dt, every) if k == 0 else s.rk3_steps_resume(Q, case.dt, every)
        dp.append(s.probe_dp(Q).cpu().numpy())
        force.append((s.marker_force() * case.markers["dV"]).sum(axis=1))
        if ((k + 1) * every) % norm_every == 0:
            norms.append([float(torch.linalg.norm(Q[c])) for c in range(case.nq)])
    s.sync()
    dp, force = np.array(dp), np.array(force)
    p_inf = case.prim_inf[4]
    d50 = np.abs(dp[:, :nprobe] - rec["dp_r50"]).max()
    d10 = np.abs(dp[:, nprobe:] - rec["dp_r10"][: dp.shape[0]]).max()
    _say(f"  WENO5-JS {steps} steps: probes max|d dp| r=50 {d50:.2e}, r=10 {d10:.2e} of p_inf {p_inf:.3f}; "
         f"force rel {_rel(force, rec['force']):.2e}; norms rel {_rel(np.array(norms), rec['norms']):.2e}")
    assert d50 <= 1e-12 * p_inf and d10 <= 1e-12 * p_inf
    assert _rel(force, rec["force"]) <= 1e-10
    assert _rel(np.array(norms), rec["norms"]) <= 1e-12
    g = Q.reshape(case.nq, -1)[:, torch.from_numpy(rec["cells"]).cuda()].cpu().numpy()
    o = rec["snaps"][-1]
    Q0s = Q0.reshape(case.nq, -1)[:, rec["cells"]]
    scale = natural_scale(case)
    for c in range(case.nq):
        rel = np.linalg.norm(g[c] - o[c]) / max(np.linalg.norm(o[c]), scale[c] * np.sqrt(o[c].size))
        d, dev = np.abs(g[c] - o[c]).max(), np.abs(o[c] - Q0s[c]).max()
        _say(f"  step {steps} component {c}: rel L2 {rel:.3e}, max|dQ| {d:.3e} of change {dev:.3e}")
        assert rel <= 1e-12
        assert d <= TOL_ELEM * dev + ELEM_ULPS * np.finfo(float).eps * scale[c], (c, d, dev)
