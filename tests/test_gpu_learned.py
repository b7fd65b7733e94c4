"""The learned TENO5 selector on the GPU, through the C ABI, against the FP64 references:

* BF16 MFMA forward and backward against the oracle network fed the same BF16-rounded values
  (FP32 accumulation order is the only difference: 1e-3 relative);
* harvested features, labels and the significance gate against the oracle's;
* the learned stage with a network that always falls back equals the FP32 precision form
  bitwise where every side is significant, and with a network that keeps every sub-stencil
  equals it in every cell whose faces TENO5 keeps whole; insignificant sides keep everything;
* a network trained on the GPU from harvested faces: loss falls, and the FP32+learned run
  matches the FP64 oracle's acoustic pressure within 1%.
"""
import time

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


@pytest.fixture(scope="module")
def mlp():
    from oracle import mlp as M

    return M


def _solver(case, **kw):
    from paper_1905_00182_amd import fsa

    return fsa.Solver(case, **kw)


def _small(n=128, precision="learned32"):
    return W.config2(n=n, h=1.0 / 16.0, sponge=2.0, nprobe=0).with_(precision=precision)


def _rand_theta(mlp, seed):
    return np.float32(mlp.init_params(seed) + 0.05 * np.random.default_rng(seed).normal(size=mlp.NPARAM)).astype(np.float64)


def _rand_feats(n, seed):
    f = np.random.default_rng(seed).uniform(-1, 1, size=(n, 16)).astype(np.float32)
    f[:, 15] = 0.0
    return f


def test_mlp_forward_matches_oracle(torch_cuda, mlp):
    s = _solver(_small())
    theta = _rand_theta(mlp, 1)
    s.mlp_set(theta)
    X = _rand_feats(1000, 2)
    zg = s.mlp_forward(torch_cuda.from_numpy(X).cuda()).cpu().numpy()
    zo, _ = mlp.forward(theta, X[:, :15].astype(np.float64), emulate=True)
    rel = np.linalg.norm(zg - zo) / np.linalg.norm(zo)
    _say("forward rel", rel)
    assert rel < 1e-3
    assert np.abs(zg - zo).max() < 1e-2 * np.abs(zo).max()


def test_bf16_parameters_set_exactly(torch_cuda, mlp):
    """fsa_set_mlp takes BF16 parameters: the FP32 master copy it keeps is their exact
    widening, and the logits equal those of fsa_mlp_set given that FP32 copy, bit for bit."""
    torch = torch_cuda
    theta = torch.from_numpy(_rand_theta(mlp, 3).astype(np.float32)).to(torch.bfloat16)
    wide = theta.to(torch.float32).numpy()
    X = torch.from_numpy(_rand_feats(500, 4)).cuda()
    a, b = _solver(_small()), _solver(_small())
    a.set_mlp_bf16(theta)
    b.mlp_set(wide)
    assert np.array_equal(a.mlp_get(), wide)
    za, zb = a.mlp_forward(X).cpu().numpy(), b.mlp_forward(X).cpu().numpy()
    assert np.array_equal(za, zb) and np.abs(za).max() > 0
    bits = theta.view(torch.int16).numpy().view(np.uint16)
    a.set_mlp_bf16(bits)                        # the same parameters as uint16 bit patterns
    assert np.array_equal(a.mlp_get(), wide)
    with pytest.raises(ValueError):
        a.set_mlp_bf16(bits[:-1])


def test_mlp_gradient_matches_oracle(torch_cuda, mlp):
    s = _solver(_small())
    theta = _rand_theta(mlp, 3)
    s.mlp_set(theta)
    X = _rand_feats(777, 4)
    Y = np.random.default_rng(5).integers(0, 8, size=777).astype(np.uint8)
    g, loss = s.mlp_grad(torch_cuda.from_numpy(X).cuda(), torch_cuda.from_numpy(Y).cuda())
    Yb = np.stack([(Y >> k) & 1 for k in range(3)], axis=1).astype(np.float64)
    lo, go = mlp.loss_and_grad(theta, X[:, :15].astype(np.float64), Yb, emulate=True)
    gg = g.cpu().numpy()
    rel = np.linalg.norm(gg - go) / np.linalg.norm(go)
    _say("loss", float(loss.item()), lo, "grad rel", rel)
    assert abs(float(loss.item()) - lo) <= 1e-5 * lo
    assert rel < 1e-3
    for name, (a, b) in {"W1": (0, 480), "W2": (512, 1536), "W3": (1568, 1664), "b": (1664, 1667)}.items():
        assert np.linalg.norm(gg[a:b] - go[a:b]) <= 2e-3 * np.linalg.norm(go[a:b]) + 1e-12, name


def test_adam_step_matches_oracle(torch_cuda, mlp):
    s = _solver(_small())
    theta = _rand_theta(mlp, 6)
    s.mlp_set(theta)
    X = _rand_feats(512, 7)
    Y = np.random.default_rng(8).integers(0, 8, size=512).astype(np.uint8)
    s.mlp_train_step(torch_cuda.from_numpy(X).cuda(), torch_cuda.from_numpy(Y).cuda(), 1e-3)
    got = s.mlp_get().astype(np.float64)
    Yb = np.stack([(Y >> k) & 1 for k in range(3)], axis=1).astype(np.float64)
    _, go = mlp.loss_and_grad(theta, X[:, :15].astype(np.float64), Yb, emulate=True)
    want, _, _ = mlp.adam(theta, np.zeros_like(theta), np.zeros_like(theta), go, 1, 1e-3)
    close = np.abs(got - want) <= 1e-3 * 1e-3 + 1e-6 * np.abs(want)
    _say("adam: fraction within 1e-3 lr:", close.mean())
    assert close.mean() > 0.99


def _bump_state(case, amp=0.02, radius=1.0, centre=(0.7, -0.4)):
    """Uniform stream plus a compactly supported cos^2 bump in rho and p and a 5% density
    step at x = 1.6 for |y| < 0.8: large regions are exactly uniform (insignificant sides)."""
    xs = W.centres(case)
    r = np.sqrt((xs[0] - centre[0]) ** 2 + (xs[1] - centre[1]) ** 2)
    b = np.where(r < radius, np.cos(0.5 * np.pi * r / radius) ** 2, 0.0)
    rho = case.prim_inf[0] * (1.0 + amp * b) * np.where((xs[0] > 1.6) & (np.abs(xs[1]) < 0.8), 1.05, 1.0)
    p = case.prim_inf[4] * (1.0 + amp * b)
    vel = [np.full(case.shape, case.prim_inf[1]), np.full(case.shape, case.prim_inf[2])]
    return W.conserved(case, rho, vel, p)


def _face_list(nx, ny):
    """(dir, i, j) of every face in the harvest order: x faces (j-major, i = -1..nx-1), then y."""
    out = [(0, i, j) for j in range(ny) for i in range(-1, nx)]
    out += [(1, i, j) for j in range(-1, ny) for i in range(nx)]
    return out


def test_harvest_matches_oracle(torch_cuda):
    from oracle.oracle import Oracle

    case = _small(n=96)
    Q0 = _bump_state(case)
    s = _solver(case)
    nx, ny = case.n[0], case.n[1]
    total = 2 * ((nx + 1) * ny + nx * (ny + 1))
    feats, labels, n = s.harvest(torch_cuda.from_numpy(Q0).cuda(), 1.0, 1, total)
    F, L = feats.cpu().numpy(), labels.cpu().numpy()
    o = Oracle(case)
    alpha = o.alpha(Q0)
    sides = [(d, i, j, sd) for (d, i, j) in _face_list(nx, ny) for sd in (0, 1)
             if o.face_significant(Q0, d, (i, j), sd)]
    _say("harvest: significant sides", len(sides), "of", total, "; GPU wrote", n)
    assert 0 < len(sides) < total // 2
    assert n == len(sides)
    rng = np.random.default_rng(9)
    cut = np.flatnonzero(L != 7)
    assert len(cut) > 20
    picks = np.concatenate([rng.choice(n, 300, replace=False), rng.choice(cut, min(200, len(cut)), replace=False)])
    bad = 0
    for k in picks:
        d, i, j, sd = sides[int(k)]
        np.testing.assert_allclose(F[k, :15], o.face_features(Q0, d, (i, j), sd), rtol=0, atol=1e-6)
        assert F[k, 15] == 0.0
        lo = o.face_label(Q0, d, (i, j), sd, alpha[d])
        if L[k] != lo:
            bad += 1
            if bad <= 12:
                _say(f"  label mismatch at dir {d} cell ({i},{j}) side {sd}: gpu {L[k]} oracle {lo}")
    _say("harvest: label mismatches", bad, "of", len(picks), "; sides with a cut-off", len(cut))
    assert bad == 0


def test_harvest3d_matches_oracle(torch_cuda):
    """3D harvest (the sphere case's pulse at 32^3): the significant sides of all three
    directions in face order, their features and labels against the oracle's."""
    from oracle.oracle import Oracle

    case = W.config3(n=32, scheme="teno5", nmark=400)
    Q0 = W.config3_state(case)
    s = _solver(case)
    nx, ny, nz = case.n
    faces = [(0, i, j, k) for k in range(nz) for j in range(ny) for i in range(-1, nx)]
    faces += [(1, i, j, k) for k in range(nz) for j in range(-1, ny) for i in range(nx)]
    faces += [(2, i, j, k) for k in range(-1, nz) for j in range(ny) for i in range(nx)]
    total = 2 * len(faces)
    feats, labels, n = s.harvest(torch_cuda.from_numpy(Q0).cuda(), 1.0, 1, total)
    F, L = feats.cpu().numpy(), labels.cpu().numpy()
    o = Oracle(case)
    alpha = o.alpha(Q0)
    sides = [(d, i, j, k, sd) for (d, i, j, k) in faces for sd in (0, 1)
             if o.face_significant(Q0, d, (i, j, k), sd)]
    _say("3D harvest: significant sides", len(sides), "of", total, "; GPU wrote", n)
    assert 0 < len(sides) < total // 2
    assert n == len(sides)
    rng = np.random.default_rng(10)
    cut = np.flatnonzero(L != 7)
    picks = np.concatenate([rng.choice(n, 300, replace=False), rng.choice(cut, min(200, len(cut)), replace=False)])
    for kk in picks:
        d, i, j, k, sd = sides[int(kk)]
        np.testing.assert_allclose(F[kk, :15], o.face_features(Q0, d, (i, j, k), sd), rtol=0, atol=1e-6)
        assert L[kk] == o.face_label(Q0, d, (i, j, k), sd, alpha[d]), (d, i, j, k, sd)
    _say("3D harvest: sides with a cut-off", len(cut))
    assert len(cut) > 20


def test_harvest_selection_is_deterministic(torch_cuda):
    case = _small(n=96)
    Q = torch_cuda.from_numpy(W.config2_noisy_state(case)).cuda()
    s = _solver(case)
    a = s.harvest(Q, 0.1, 7, 200000)
    b = s.harvest(Q, 0.1, 7, 200000)
    assert a[2] == b[2] and torch_cuda.equal(a[0], b[0]) and torch_cuda.equal(a[1], b[1])
    assert (a[1] != 7).sum().item() > 0


def _const_net(mlp, logit):
    theta = np.zeros(mlp.NPARAM)
    theta[1664:1667] = logit
    return theta


def test_insignificant_sides_keep_everything(torch_cuda, mlp):
    from oracle.oracle import Oracle

    case = _small(n=96)
    Q0 = _bump_state(case)
    sl = _solver(case)
    sl.mlp_set(_const_net(mlp, -10.0), 0.8)          # every significant side falls back
    fx, fy = sl.face_flags(torch_cuda.from_numpy(Q0).cuda())
    sl.sync()
    st = sl.stats()
    fx, fy = fx.cpu().numpy().view(np.uint32), fy.cpu().numpy().view(np.uint32)
    o = Oracle(case)
    nx, ny = case.n[0], case.n[1]
    nsig = 0
    for d, i, j in _face_list(nx, ny):
        s0 = o.face_significant(Q0, d, (i, j), 0)
        s1 = o.face_significant(Q0, d, (i, j), 1)
        nsig += int(s0) + int(s1)
        word = fx[j, i + 1] if d == 0 else fy[j + 1, i]
        if not s0:
            assert word & 0xFFFF == 0x0FFF, (d, i, j)
        if not s1:
            assert word >> 16 == 0x0FFF, (d, i, j)
    _say("flags: significant sides", st.significant_sides, "oracle", nsig, "of", st.learned_sides)
    assert st.significant_sides == nsig == st.fallback_sides
    assert st.learned_sides == 2 * ((nx + 1) * ny + nx * (ny + 1))


def test_learned_fallback_equals_precision_form(torch_cuda, mlp):
    case = _small(n=160)
    Q0 = W.config2_noisy_state(case)
    Q0[0, 60:80, 40:90] *= 1.04
    Q = torch_cuda.from_numpy(Q0).cuda()
    s32 = _solver(case.with_(precision="mixed32"))
    L32 = s32.rhs(Q)
    sl = _solver(case)
    sl.mlp_set(_const_net(mlp, -10.0), 0.8)          # predicts no sub-stencil: every side falls back
    Ll = sl.rhs(Q)
    sl.sync()
    st = sl.stats()
    _say("fallback test: sides", st.learned_sides, "significant", st.significant_sides, "fallback", st.fallback_sides)
    assert st.fallback_sides == st.significant_sides == st.learned_sides > 0
    assert torch_cuda.equal(L32, Ll)


def test_learned_keep_all_equals_precision_form_where_teno_keeps_all(torch_cuda, mlp):
    case = W.periodic_box(dim=2, n=128, scheme="teno5", mu=0.002).with_(precision="learned32")
    Q0 = W.perturbed_state(case, seed=11, amp=1e-3)
    Q = torch_cuda.from_numpy(Q0).cuda()
    # the precision form's own TENO5 decisions: a network that always falls back
    sf = _solver(case)
    sf.mlp_set(_const_net(mlp, -10.0), 0.8)
    fx, fy = sf.face_flags(Q)
    sf.sync()
    assert sf.stats().significant_sides == sf.stats().learned_sides
    keep = 0x0FFF0FFF
    fx, fy = fx.cpu().numpy().view(np.uint32), fy.cpu().numpy().view(np.uint32)
    whole = (fx[:, :-1] == keep) & (fx[:, 1:] == keep) & (fy[:-1, :] == keep) & (fy[1:, :] == keep)
    sl = _solver(case)
    sl.mlp_set(_const_net(mlp, 10.0), 0.8)           # confident: keep every sub-stencil
    gx, gy = sl.face_flags(Q)
    assert torch_cuda.all(gx == keep) and torch_cuda.all(gy == keep)
    Ll = sl.rhs(Q).cpu().numpy()
    s32 = _solver(case.with_(precision="mixed32"))
    L32 = s32.rhs(Q).cpu().numpy()
    _say("cells whose four faces TENO5 keeps whole:", int(whole.sum()), "of", whole.size)
    assert whole.sum() > 0.5 * whole.size
    assert np.array_equal(Ll[:, whole], L32[:, whole])
    assert not np.array_equal(Ll, L32)


@pytest.fixture(scope="module")
def trained(torch_cuda, mlp):
    """A selector trained on the GPU (the library's training procedure) from the significant
    face sides of FP64 runs of the scattering case (TENO5) and the rotating-cylinder
    miniature (uniform start)."""
    from paper_1905_00182_amd import selector

    cases = selector.training_cases()
    F, L = selector.harvest(cases)
    ncut = int((L != 7).sum().item())
    _say("harvested", F.shape[0], "significant sides;", ncut, "with a cut sub-stencil")
    theta, losses = selector.train(F, L)
    _say("training loss", [round(x, 5) for x in losses])
    tr = _solver(_small())
    tr.mlp_set(theta, 0.8)
    z = tr.mlp_forward(F).cpu().numpy()
    bits = (z[:, 0] > 0) | ((z[:, 1] > 0) << 1) | ((z[:, 2] > 0) << 2)
    conf = np.abs(z).min(axis=1) >= np.log(9.0)        # |2 sigma - 1| >= 0.8
    Lh = L.cpu().numpy()
    acc = np.mean(bits == Lh)
    accc = np.mean(bits[conf] == Lh[conf])
    _say(f"training-set accuracy {acc:.4f}; confident {conf.mean():.3f} of sides, accuracy there {accc:.4f}")
    return {"theta": theta, "losses": losses, "acc": acc, "conf": conf.mean(), "accc": accc,
            "c1": cases[0][0], "c2": cases[1][0]}


def test_training_reduces_loss(trained):
    assert trained["losses"][-1] < 0.2 * trained["losses"][0]
    assert trained["conf"] > 0.6 and trained["accc"] > 0.95


def _learned_vs_oracle(torch, case, Q0, theta, nsteps, stride=1):
    from oracle.oracle import Oracle

    o = Oracle(case)
    Qo = Q0.copy()
    dpo = []
    for _ in range(nsteps):
        o.rk3_step(Qo, case.dt)
        dpo.append(o.probe_dp(Qo))
    dpo = np.array(dpo)
    res = {}
    for prec in ("mixed32", "learned32"):
        sv = _solver(case.with_(precision=prec, extra={"selector_stride": stride}))
        if prec == "learned32":
            sv.mlp_set(theta, 0.8)
        Q = torch.from_numpy(Q0.copy()).cuda()
        dp = []
        for _ in range(nsteps):
            sv.rk3_step(Q, case.dt)
            dp.append(sv.probe_dp(Q).cpu().numpy())
        sv.sync()
        dp = np.array(dp)
        st = sv.stats()
        n = max(st.learned_sides, 1)
        res[prec] = (np.linalg.norm(dp - dpo) / np.linalg.norm(dpo), st.significant_sides / n, st.fallback_sides / n)
    _say(f"{case.name} {case.n[:2]}, {nsteps} steps, selector stride {stride}: e_p precision form {res['mixed32'][0]:.3e}, "
         f"learned {res['learned32'][0]:.3e} (significant {res['learned32'][1]:.4f}, fallback "
         f"{res['learned32'][2]:.4f} of face sides); probe |dp| up to {np.abs(dpo).max():.2e}")
    return res


@pytest.mark.parametrize("stride", [1, 3])
def test_learned_acoustic_error_config1_held_out(torch_cuda, trained, stride):
    """Config 1 with the pulse moved to (-1.5, 1.0): a run the selector was not trained on."""
    c = trained["c1"]
    res = _learned_vs_oracle(torch_cuda, c, W.pulse_state(c, (-1.5, 1.0)), trained["theta"], c.steps, stride)
    assert res["learned32"][0] < 1e-2
    assert res["mixed32"][0] < 1e-5


@pytest.mark.parametrize("stride", [1, 3])
def test_learned_acoustic_error_config2_small(torch_cuda, trained, stride):
    """A 256^2 miniature of the rotating-cylinder case (the selector was trained on the full
    case), 150 steps from the uniform start."""
    c = W.config2(n=256, h=1.0 / 16.0, sponge=2.0, nprobe=48, rprobe=3.0)
    res = _learned_vs_oracle(torch_cuda, c, W.config2_state(c), trained["theta"], 150, stride)
    assert res["learned32"][0] < 1e-2


def test_network_gain_over_plain_teno(torch_cuda, trained):
    """What the trained network gains over the method without it, on the 2048^2 rotating
    cylinder (800 steps from the uniform start): with the selector once per step, plain TENO5
    is evaluated on under a tenth of the face sides (the fallback ones) instead of all, and
    the step takes at most 0.85 of the precision form's (plain FP32 TENO5) time, with the
    far-field probe pressure (a ring of radius 10, which the start-up wave crosses) within 1%
    of the FP64 run's (itself the oracle's: the parity tests)."""
    torch = torch_cuda
    c = W.config2(nprobe=64, rprobe=10.0)
    Q0 = torch.from_numpy(W.config2_state(c)).cuda()
    out = {}
    for name, prec, stride in (("fp64", "fp64", 1), ("mixed32", "mixed32", 1), ("learned32", "learned32", 3)):
        sv = _solver(c.with_(precision=prec, extra={"selector_stride": stride}))
        if prec == "learned32":
            sv.mlp_set(trained["theta"], 0.8)
        Q = Q0.clone()
        sv.rk3_steps(Q, c.dt, 3)                  # warm-up (segment tuning)
        Q = Q0.clone()
        sv.set_state(None, 0.0, 0)
        st0 = sv.stats()
        dps = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(80):
            sv.rk3_steps(Q, c.dt, 10)
            dps.append(sv.probe_dp(Q))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = sv.stats()
        n = max(st.learned_sides - st0.learned_sides, 1)
        out[name] = (wall, torch.stack(dps), (st.fallback_sides - st0.fallback_sides) / n)
        sv.close()
    e_p = float(torch.linalg.norm(out["learned32"][1] - out["fp64"][1]) / torch.linalg.norm(out["fp64"][1]))
    ratio = out["learned32"][0] / out["mixed32"][0]
    _say(f"network gain: learned (stride 3) {out['learned32'][0] * 1e3 / 800:.3f} ms/step vs plain FP32 TENO5 "
         f"{out['mixed32'][0] * 1e3 / 800:.3f} (ratio {ratio:.3f}), FP64 {out['fp64'][0] * 1e3 / 800:.3f}; fallback "
         f"{out['learned32'][2]:.4f} of sides; e_p vs FP64 {e_p:.3e} (|dp| up to "
         f"{float(out['fp64'][1].abs().max()):.2e})")
    assert float(out["fp64"][1].abs().max()) > 1e-5
    assert out["learned32"][2] < 0.1
    assert ratio < 0.85
    assert e_p < 1e-2


@pytest.mark.parametrize("stride", [1, 3])
def test_quiet_tiles_change_nothing(torch_cuda, trained, stride):
    """The flags pass writes all-kept words for tiles whose covering stage-kernel strips spread
    by no more than the significance thresholds, without loading the state; the run must be
    bit for bit the one that evaluates every tile (FSA_NO_QUIET_TILES=1)."""
    import os

    c = trained["c2"].with_(precision="learned32", extra={"selector_stride": stride})
    Q0 = torch_cuda.from_numpy(W.config2_state(c)).cuda()
    out = []
    for off in ("0", "1"):
        os.environ["FSA_NO_QUIET_TILES"] = off
        try:
            s = _solver(c)
        finally:
            del os.environ["FSA_NO_QUIET_TILES"]
        s.mlp_set(trained["theta"], 0.8)
        Q = Q0.clone()
        s.rk3_steps(Q, c.dt, 40)
        s.rk3_steps(Q, c.dt, 20)
        s.sync()
        st = s.stats()
        out.append((Q, st.significant_sides, st.fallback_sides, st.learned_sides))
        s.close()
    _say("quiet tiles, stride", stride, ": significant / fallback / sides", out[0][1:], "vs", out[1][1:])
    assert out[0][1:] == out[1][1:]
    assert torch_cuda.equal(out[0][0], out[1][0])


@pytest.mark.parametrize("precision,stride", [("fp64", 1), ("learned32", 1), ("learned32", 3)])
def test_resume_equals_one_call(torch_cuda, trained, precision, stride):
    """Steps continued one call at a time (fsa_rk3_steps_resume: the wave speeds and quiet-tile
    ranges of the state taken from the kernels that wrote it) are bit for bit the steps of one
    call, on the rotating-cylinder miniature (markers, sponge, learned selector)."""
    c = trained["c2"].with_(precision=precision, extra={"selector_stride": stride})
    Q0 = torch_cuda.from_numpy(W.config2_state(c)).cuda()
    out = []
    for resume in (False, True):
        s = _solver(c)
        if precision == "learned32":
            s.mlp_set(trained["theta"], 0.8)
        Q = Q0.clone()
        if resume:
            s.rk3_step(Q, c.dt)
            for _ in range(29):
                s.rk3_steps_resume(Q, c.dt)
        else:
            s.rk3_steps(Q, c.dt, 30)
        s.sync()
        st = s.stats()
        out.append((Q, st.significant_sides, st.fallback_sides, st.learned_sides))
        s.close()
    _say(precision, "stride", stride, ": resumed one step at a time vs one call of 30 steps;",
         "significant / fallback / sides", out[1][1:], "vs", out[0][1:])
    assert out[0][1:] == out[1][1:]
    assert torch_cuda.equal(out[0][0], out[1][0])
