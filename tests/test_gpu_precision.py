"""The FP32 precision form (face reconstruction and viscous fluxes in FP32 on deviations from
the far field, FP64 state, RK3 and sources) against the FP64 CPU oracle, through the C ABI.

Tolerance of one right-hand side: the FP32 windows carry d = f - f_inf rounded once (relative
2^-24), each face value is a weighted sum of five of them (~30 roundings of size eps32 |d|),
so max |L32 - L64| <= 1e-5 * Sd with Sd = 2 alpha max|Q - Q_inf| / h + max|F - F_inf| / h
(eps32 = 6e-8; ~160 eps32 of margin).  Over a run the acoustic-pressure error at the probes
e_p = ||dp32 - dp64||_2 / ||dp64||_2 over probes x steps is reported and bounded by 1%.
"""
import math

import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _say(*a):
    print("[gpu]", *a, flush=True)


def _dev_scale(case, Q, alpha):
    Qinf = W.uniform_state(case)
    dq = np.abs(Q - Qinf).max()
    return 4.0 * max(alpha[: case.dim]) * dq / case.h


@pytest.mark.parametrize("scheme", ["weno5js", "teno5"])
def test_mixed32_rhs(torch_cuda, scheme):
    from oracle.oracle import Oracle
    from paper_1905_00182_amd import fsa

    case = W.config2(n=200, h=1.0 / 16.0, sponge=2.0, nprobe=0).with_(scheme=scheme)
    Q0 = W.config2_noisy_state(case)
    Q0[0, 60:80, 90:120] *= 1.02
    _say("mixed32 rhs", scheme, case.n)
    s = fsa.Solver(case.with_(precision="mixed32"))
    L32 = s.rhs(torch_cuda.from_numpy(Q0).cuda())
    s.sync()
    o = Oracle(case)
    L64 = o.rhs(Q0)
    Sd = _dev_scale(case, Q0, o.alpha(Q0))
    err = np.abs(L32.cpu().numpy() - L64).max()
    _say("  max |L32 - L64| / Sd =", err / Sd, " max|L| / Sd =", np.abs(L64).max() / Sd)
    assert err <= 1e-5 * Sd


def _probe_run(torch, case, nsteps):
    from oracle.oracle import Oracle
    from paper_1905_00182_amd import fsa

    Q0 = W.config1_state(case) if case.name.startswith("c1") else W.config2_state(case)
    s = fsa.Solver(case.with_(precision="mixed32"))
    Qg = torch.from_numpy(Q0.copy()).cuda()
    o = Oracle(case)
    Qo = Q0.copy()
    dpg, dpo = [], []
    for _ in range(nsteps):
        s.rk3_step(Qg, case.dt)
        dpg.append(s.probe_dp(Qg).cpu().numpy())
        o.rk3_step(Qo, case.dt)
        dpo.append(o.probe_dp(Qo))
    s.sync()
    dpg, dpo = np.array(dpg), np.array(dpo)
    ep = np.linalg.norm(dpg - dpo) / np.linalg.norm(dpo)
    qrel = np.linalg.norm(Qg.cpu().numpy() - Qo) / np.linalg.norm(Qo)
    return ep, qrel, np.abs(dpo).max()


def test_mixed32_acoustic_error_config1(torch_cuda):
    case = W.config1(n=128)
    ep, qrel, amp = _probe_run(torch_cuda, case, case.steps)
    _say(f"C1 mixed32, {case.steps} steps: e_p = {ep:.3e} (probe |dp| up to {amp:.2e}), state rel L2 {qrel:.2e}")
    assert amp > 1e-6
    assert ep < 1e-2


def test_mixed32_acoustic_error_config2_small(torch_cuda):
    # uniform start: the cylinder's start-up wave reaches the radius-3 probes after ~90 steps
    case = W.config2(n=256, h=1.0 / 16.0, sponge=2.0, nprobe=48, rprobe=3.0)
    ep, qrel, amp = _probe_run(torch_cuda, case, 150)
    _say(f"C2 (256^2) mixed32, 150 steps: e_p = {ep:.3e} (probe |dp| up to {amp:.2e}), state rel L2 {qrel:.2e}")
    assert ep < 1e-2
