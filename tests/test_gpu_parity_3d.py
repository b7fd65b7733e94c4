"""GPU parity of the 3D HIP path (stress pass + stage pass) against the FP64 CPU oracle, through
the C ABI, with the tolerances of the 2D tests: one right-hand side max |dL| <= 1e-13 S, after
steps the whole-state and per-component relative L2 <= 1e-12.  The sphere scattering case is
checked in a miniature over many steps and at its full 256^3 size over one step (both
schemes); the precision form at 384^3 on sampled cells and, for its acoustic error, on a
miniature of the same set-up.
"""
import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

from test_gpu_parity_2d import TENO_TIE_ELEM, TENO_TIE_TOL, _assert_q_close, _compare_rhs, _oracle, _say, _solver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _box3(scheme, n=(22, 18, 14), mu=0.004, terms=W.TERMS_ALL):
    c = W.periodic_box(dim=3, n=n[0], scheme=scheme, mu=mu, terms=terms)
    return c.with_(n=tuple(n))


@pytest.mark.parametrize("scheme", ["weno5js", "teno5"])
def test_rhs3d_periodic_ragged(torch_cuda, scheme):
    case = _box3(scheme)
    Q0 = W.perturbed_state(case, seed=31, amp=2e-2, step_amp=0.3)
    _, Lo = _compare_rhs(torch_cuda, case, Q0)
    assert np.abs(Lo).max() > 0


@pytest.mark.parametrize("term", ["conv_x", "conv_y", "conv_z", "visc", "sponge"])
def test_rhs3d_single_terms(torch_cuda, term):
    case = _box3("teno5", terms=W.TERM[term])
    case = case.with_(bc=(("extrap", "extrap"), ("extrap", "extrap"), ("extrap", "extrap")),
                      sponge_width=((0.2, 0.1), (0.15, 0.25), (0.1, 0.2)), sponge_sigma=4.0)
    Q0 = W.perturbed_state(case, seed=32, amp=2e-2, step_amp=0.3)
    _compare_rhs(torch_cuda, case, Q0)


@pytest.mark.parametrize("xhi", ["periodic", "extrap", "inflow", "nonreflect"])
def test_rhs3d_last_x_face_column(torch_cuda, xhi):
    """A grid whose n_x is a multiple of 64 takes its last x face column (x = n_x) from a
    kernel of its own: the right-hand side against the oracle with each boundary kind on the
    x+ side behind that column (component-wise TENO5, and characteristic-wise WENO5-JS)."""
    case = _box3("teno5", n=(64, 10, 8))
    lo = "periodic" if xhi == "periodic" else "extrap"
    case = case.with_(bc=((lo, xhi), ("periodic", "periodic"), ("periodic", "periodic")),
                      prim_inf=(1.0, 0.2, -0.1, 0.05, 1.0 / 1.4), inflow_amp=2e-5)
    Q0 = W.perturbed_state(case, seed=35, amp=2e-2, step_amp=0.3)
    _compare_rhs(torch_cuda, case, Q0)
    _compare_rhs(torch_cuda, case.with_(scheme="weno5js", variables="characteristic"), Q0)


def test_rhs3d_inflow_and_markers(torch_cuda):
    # inflow with the seeded perturbation on x-, zero-gradient elsewhere, sponge, a sphere
    case = W.config3(n=32, scheme="teno5", nmark=600, L=4.0).with_(
        bc=(("inflow", "extrap"), ("extrap", "extrap"), ("extrap", "extrap")),
        prim_inf=(1.0, 0.2, 0.0, 0.0, 1.0 / 1.4), inflow_amp=2e-5)
    Q0 = W.perturbed_state(case, seed=33, amp=1e-2, step_amp=0.2)
    _compare_rhs(torch_cuda, case, Q0)


def test_free_stream3d_exactly_zero(torch_cuda):
    case = W.periodic_box(dim=3, n=20, scheme="teno5", mu=0.003,
                          prim_inf=(1.0, 0.2, -0.1, 0.05, 1.0 / 1.4)).with_(n=(20, 16, 12))
    s = _solver(case)
    L = s.rhs(torch_cuda.from_numpy(W.uniform_state(case)).cuda())
    s.sync()
    assert torch_cuda.count_nonzero(L).item() == 0


def test_mass_conserved3d(torch_cuda):
    case = _box3("teno5", n=(24, 20, 16))
    Q0 = W.perturbed_state(case, seed=34, amp=2e-2, step_amp=0.3)
    s = _solver(case)
    Q = torch_cuda.from_numpy(Q0.copy()).cuda()
    s.rk3_steps(Q, case.dt, 20)
    s.sync()
    m0, m1 = Q0[0].sum(), Q[0].sum().item()
    _say("3D periodic: mass drift", (m1 - m0) / m0)
    assert abs(m1 - m0) <= 1e-13 * abs(m0)


def _steps3(torch, case, Q0, nsteps):
    _say("steps", case.name, case.n, case.scheme, case.precision, "x", nsteps)
    s = _solver(case)
    Qg = torch.from_numpy(Q0.copy()).cuda()
    s.rk3_steps(Qg, case.dt, nsteps)
    s.sync()
    o = _oracle(case)
    Qo = Q0.copy()
    for _ in range(nsteps):
        o.rk3_step(Qo, case.dt)
    return s, o, Qg, Qo


def test_rhs3d_periodic_source(torch_cuda):
    """The periodic Gaussian pressure source (Sec. 3) with every other term on, at a time that is
    not a multiple of its period: one right-hand side against the oracle."""
    case = _box3("teno5").with_(src_amp=0.01, src_b=16.0, src_omega=2.0 * np.pi, src_x=(0.41, 0.37, 0.33))
    Q0 = W.perturbed_state(case, seed=31, amp=1e-2, step_amp=0.3)
    t = 0.37
    _say("rhs periodic source at t =", t)
    s = _solver(case)
    s.set_state(None, t, 0)
    Lg = s.rhs(torch_cuda.from_numpy(Q0).cuda())
    s.sync()
    Lg = Lg.cpu().numpy()
    o = _oracle(case)
    o.set_state(None, t, 0)
    Lo = o.rhs(Q0)
    S = 2.0 * np.abs(Q0).max() * max(o.alpha(Q0)[:3]) / case.h
    err = np.abs(Lg - Lo).max()
    _say("  max |dL| / S =", err / S)
    assert err <= 1e-13 * S
    # the source is a visible part of the energy equation here
    o0 = _oracle(case.with_(src_amp=0.0))
    assert np.abs(Lo[4] - o0.rhs(Q0)[4]).max() > 1e-3 / (W.GAMMA - 1.0)


def test_rk3_config3_source_miniature(torch_cuda):
    """The sphere case driven by the periodic source from a quiescent start (the stage times
    t, t + dt, t + dt/2 enter through the source), against the oracle: WENO5-JS over 30 steps
    (about four periods of the source) to 1e-12; TENO5 over one step to 1e-12 (over many steps
    its cut-off decides on the rounding noise of the quiescent far field, as on the pulse)."""
    case = W.config3_source(n=48, scheme="weno5js", nmark=2000)
    Q0 = W.uniform_state(case)
    s, o, Qg, Qo = _steps3(torch_cuda, case, Q0, 30)
    _assert_q_close(Qg.cpu().numpy(), Qo, Q0, case)
    # without the source the quiescent state stays exactly as it is
    assert np.abs(Qo[4] - Q0[4]).max() > 1e-7
    np.testing.assert_allclose(s.marker_force(), o.marker_force(), rtol=1e-9, atol=1e-12)
    case = case.with_(scheme="teno5")
    s, o, Qg, Qo = _steps3(torch_cuda, case, Q0, 1)
    _assert_q_close(Qg.cpu().numpy(), Qo, Q0, case)


def test_source_rejected_in_2d(torch_cuda):
    from paper_1905_00182_amd import fsa

    case = W.periodic_box(dim=2, n=16).with_(src_amp=0.01)
    with pytest.raises(fsa.FsaError):
        fsa.Solver(case)


def test_rk3_config3_miniature_weno(torch_cuda):
    case = W.config3(n=48, scheme="weno5js", nmark=2000)
    Q0 = W.config3_state(case)
    s, o, Qg, Qo = _steps3(torch_cuda, case, Q0, 30)
    _assert_q_close(Qg.cpu().numpy(), Qo, Q0, case)
    np.testing.assert_allclose(s.marker_force(), o.marker_force(), rtol=1e-9, atol=1e-12)


def test_rk3_config3_miniature_teno_smooth_state(torch_cuda):
    """TENO5 with the sphere over 30 steps on a state whose every region varies well above
    rounding (seeded smooth modes of relative size 1e-3): the decisions are robust and the
    1e-12 bound holds."""
    case = W.config3(n=48, scheme="teno5", nmark=2000)
    Q0 = W.perturbed_state(case, seed=35, amp=1e-3)
    s, o, Qg, Qo = _steps3(torch_cuda, case, Q0, 30)
    _assert_q_close(Qg.cpu().numpy(), Qo, Q0, case)
    np.testing.assert_allclose(s.marker_force(), o.marker_force(), rtol=1e-9, atol=1e-12)


def test_rk3_config3_miniature_teno_pulse(torch_cuda):
    """TENO5 on the pulse state: one step to 1e-12 in relative L2; 30 steps to the tie bounds
    (TENO_TIE_*: the decisions are checked on the same run's stage inputs in
    test_gpu_teno_ties.py), with the probe pressure to 1e-6 of its amplitude."""
    case = W.config3(n=48, scheme="teno5", nmark=2000)
    Q0 = W.config3_state(case)
    s, o, Qg, Qo = _steps3(torch_cuda, case, Q0, 1)
    _assert_q_close(Qg.cpu().numpy(), Qo, Q0, case, tol_elem=TENO_TIE_ELEM)
    s, o, Qg, Qo = _steps3(torch_cuda, case, Q0, 30)
    _assert_q_close(Qg.cpu().numpy(), Qo, Q0, case, tol=TENO_TIE_TOL, tol_elem=TENO_TIE_ELEM)
    dpg = s.probe_dp(Qg).cpu().numpy()
    dpo = o.probe_dp(Qo)
    _say(f"  probes: max |dp_gpu - dp_ora| = {np.abs(dpg - dpo).max():.3e} of amplitude {np.abs(dpo).max():.3e}")
    assert np.abs(dpg - dpo).max() <= 1e-6 * np.abs(dpo).max()


@pytest.mark.parametrize("scheme", ["teno5", "weno5js"])
def test_config3_full_size(torch_cuda, scheme):
    """The 256^3 sphere case with 10^4 markers, one step, whole state against the oracle
    (relative L2 1e-12; TENO5 element-wise to the tie bound: a tie in the pulse's far tail,
    where the signal is 1e-11 of the state, already decides differently in one step)."""
    case = W.config3(n=256, scheme=scheme)
    Q0 = W.config3_state(case)
    s, o, Qg, Qo = _steps3(torch_cuda, case, Q0, 1)
    if scheme == "teno5":
        _assert_q_close(Qg.cpu().numpy(), Qo, Q0, case, tol_elem=TENO_TIE_ELEM)
    else:
        _assert_q_close(Qg.cpu().numpy(), Qo, Q0, case)


def test_precision3d_rhs_config4_full_size_sampled(torch_cuda):
    """The 384^3 precision form: one right-hand side on 4000 sampled cells (anywhere, around the
    pulse and the sphere's support, next to the boundaries) against the FP64 oracle, within the FP32 bound of the
    2D precision tests (1e-5 of the deviation scale)."""
    case = W.config4(n=384)
    Q0 = W.config3_state(case)
    s = _solver(case)
    L = s.rhs(torch_cuda.from_numpy(Q0).cuda())
    s.sync()
    o = _oracle(case)
    rng = np.random.default_rng(7)
    n = case.n[0]
    pts = [rng.integers(0, n, size=(2000, 3))]
    c = n // 2
    pts.append(rng.integers(c - 12, c + 12, size=(600, 3)))                # around the sphere
    ip = int(round((2.0 - case.lo[0]) / case.h))                              # around the pulse
    pts.append(np.stack([rng.integers(ip - 12, ip + 12, 1000), rng.integers(c - 12, c + 12, 1000),
                         rng.integers(c - 12, c + 12, 1000)], 1))
    pts.append(np.stack([rng.integers(0, n, 400), rng.integers(0, n, 400), rng.choice([0, 1, n - 2, n - 1], 400)], 1))
    ijk = np.concatenate(pts)
    lin = (ijk[:, 2] * n + ijk[:, 1]) * n + ijk[:, 0]
    Lo = o.rhs_cells(Q0, lin)
    Lg = L.reshape(case.nq, -1)[:, torch_cuda.from_numpy(lin).cuda()].cpu().numpy()
    alpha = o.alpha(Q0)
    dq = np.abs(Q0 - W.uniform_state(case)).max()
    Sd = 4.0 * max(alpha) * dq / case.h
    err = np.abs(Lg - Lo).max()
    _say(f"384^3 precision form rhs on {lin.size} cells: max|dL| / Sd = {err / Sd:.3e}; max|L| / Sd = {np.abs(Lo).max() / Sd:.3e}")
    assert np.abs(Lo).max() > 1e-2 * Sd          # the samples reach the pulse
    assert err <= 1e-5 * Sd


def test_precision3d_acoustic_error(torch_cuda):
    """Precision form of the sphere case (miniature, 64 probes on r = 4): acoustic pressure
    against the FP64 oracle over the run, e_p = ||dp32 - dp64|| / ||dp64|| < 1%."""
    case = W.config3(n=64, scheme="teno5", nmark=2000).with_(precision="mixed32")
    Q0 = W.config3_state(case)
    nsteps, every = 100, 5
    s = _solver(case)
    o = _oracle(case)
    Qg = torch_cuda.from_numpy(Q0.copy()).cuda()
    Qo = Q0.copy()
    dpg, dpo = [], []
    for _ in range(nsteps // every):
        s.rk3_steps(Qg, case.dt, every)
        dpg.append(s.probe_dp(Qg).cpu().numpy())
        for _ in range(every):
            o.rk3_step(Qo, case.dt)
        dpo.append(o.probe_dp(Qo))
    dpg, dpo = np.array(dpg), np.array(dpo)
    ep = np.linalg.norm(dpg - dpo) / np.linalg.norm(dpo)
    _say(f"3D precision form, 64^3, {nsteps} steps: e_p = {ep:.3e} (probe |dp| up to {np.abs(dpo).max():.2e})")
    assert np.abs(dpo).max() > 1e-7
    assert ep < 1e-2
