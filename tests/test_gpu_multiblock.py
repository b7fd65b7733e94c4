"""One domain in several blocks on one GPU (fsa_mb_*): slabs along the last direction, each
a context over its layers and FSA_HALO halo layers placed in the global grid. After every
stage, explicit halo copies run and the wave speeds are maximised across blocks. This is
the one-GPU stand-in for the paper's domain decomposition across processes (Sec. 2).

The blocks' result must equal one context's over the whole domain bit for bit. The cases
are the rotating-cylinder set-up with inflow noise, sponge and markers (2D, blocks along y),
a periodic box whose halos wrap around (2D), the sphere with its markers (3D, blocks along
z), with uneven block sizes, and markers that move from block to block.
"""
import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

from test_gpu_parity_2d import _say, _solver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _single_and_blocks(torch, case, Q0, nblocks, nsteps):
    from paper_1905_00182_amd import fsa

    s = _solver(case)
    Qs = torch.from_numpy(Q0.copy()).cuda()
    s.rk3_steps(Qs, case.dt, nsteps)
    s.sync()
    m = fsa.MultiBlock(case, nblocks)
    m.scatter(torch.from_numpy(Q0.copy()).cuda())
    m.rk3_steps(case.dt, nsteps)
    Qm = m.gather()
    torch.cuda.synchronize()
    info = [m.block_info(b) for b in range(nblocks)]
    _say(f"{case.name} {case.n[:case.dim]} in {nblocks} blocks (first, layers, halo below, above): {info}")
    return s, m, Qs.cpu().numpy(), Qm.cpu().numpy(), info


def _assert_bitwise(Qs, Qm, Q0):
    diff = np.argwhere(Qs != Qm)
    assert diff.size == 0, f"{diff.shape[0]} cells differ, first {diff[:4].tolist()}, " \
                           f"max |d| {np.abs(Qs - Qm).max():.3e}"
    assert np.abs(Qs - Q0).max() > 0.0


def test_rotating_cylinder_four_blocks(torch_cuda):
    case = W.config2(n=256, h=1.0 / 16.0, sponge=2.0, nprobe=8, rprobe=4.0)
    Q0 = W.config2_noisy_state(case)
    s, m, Qs, Qm, info = _single_and_blocks(torch_cuda, case, Q0, 4, 20)
    assert [i[1] for i in info] == [64, 64, 64, 64] and info[0][2] == 0 and info[-1][3] == 0
    _assert_bitwise(Qs, Qm, Q0)
    Fs, Fm = s.marker_force(), m.marker_force()
    assert np.array_equal(Fs, Fm)


def test_rotating_cylinder_uneven_blocks_teno_and_weno(torch_cuda):
    for scheme, nb in (("teno5", 7), ("weno5js", 3)):
        case = W.config2(n=200, h=1.0 / 16.0, sponge=2.0, nprobe=8, rprobe=4.0).with_(n=(180, 203, 1), scheme=scheme)
        Q0 = W.config2_noisy_state(case)
        Q0[0, 90:120, 60:80] *= 1.05
        s, m, Qs, Qm, info = _single_and_blocks(torch_cuda, case, Q0, nb, 12)
        assert sum(i[1] for i in info) == 203
        _assert_bitwise(Qs, Qm, Q0)
        assert np.array_equal(s.marker_force(), m.marker_force())


def test_periodic_box_wrapped_halos(torch_cuda):
    case = W.periodic_box(dim=2, n=120, scheme="teno5", mu=0.004).with_(n=(120, 90, 1))
    Q0 = W.perturbed_state(case, seed=51, amp=2e-2, step_amp=0.3)
    s, m, Qs, Qm, info = _single_and_blocks(torch_cuda, case, Q0, 3, 10)
    assert all(i[2] == 4 and i[3] == 4 for i in info)
    _assert_bitwise(Qs, Qm, Q0)


def _blocks_reached(X, case, info):
    """For each marker, the set of blocks whose own layers its 4-point support reaches."""
    d = case.dim - 1
    j0 = np.floor((X[d] - case.lo[d]) / case.h - 0.5).astype(int) - 1
    return [frozenset(b for b, (first, count, _, _) in enumerate(info) if j + 3 >= first and j <= first + count - 1)
            for j in j0]


@pytest.mark.parametrize("what", ["plate", "insect"])
def test_moving_markers_cross_blocks(torch_cuda, what):
    """EXTERNAL markers moved every step on both sides: the rigid flapping plate (its motion
    played 40 times faster, so that it heaves through the block boundary at y = 0 in 60 steps)
    in 4 blocks (24 steps re-deal markers) and the hovering insect's wings in 5 uneven blocks
    (3 steps). The markers whose supports
    come to reach another set of blocks are dealt out again with their penalty integrals; the
    state and marker forces must stay equal to one context's bit for bit."""
    from paper_1905_00182_amd import fsa

    torch = torch_cuda
    if what == "plate":
        case, nb, nsteps, least = W.config5(n=128, L=8.0, nmark=128), 4, 60, 10
        kin = lambda n: (W.plate_kinematics(case, 40.0 * n * case.dt)[0],
                         W.plate_kinematics(case, 40.0 * n * case.dt)[1])
    else:
        case, nb, nsteps, least = W.insect(n=192, L=3.84, sponge=0.5, nprobe=0), 5, 40, 2
        kin = lambda n: W.insect_kinematics(case, n * case.dt)
    Q0 = W.uniform_state(case)
    s = _solver(case)
    m = fsa.MultiBlock(case, nb)
    info = [m.block_info(b) for b in range(nb)]
    Qs = torch.from_numpy(Q0.copy()).cuda()
    m.scatter(torch.from_numpy(Q0.copy()).cuda())
    deals, redealt = [], 0
    for n in range(nsteps):
        X, U = kin(n)
        deal = _blocks_reached(X, case, info)
        redealt += int(bool(deals) and deal != deals[-1])
        deals.append(deal)
        s.set_marker_kinematics(X, U)
        m.set_marker_kinematics(X, U)
        s.rk3_step(Qs, case.dt) if n == 0 else s.rk3_steps_resume(Qs, case.dt)
        m.rk3_steps(case.dt, 1)
    Qm = m.gather()
    torch.cuda.synchronize()
    crossing = sum(len(d) > 1 for d in deals[-1])
    _say(f"{what} in {nb} blocks: {redealt} of {nsteps - 1} steps dealt markers out again; "
         f"{crossing} markers reach two blocks at the end")
    assert redealt >= least
    Qs, Qm = Qs.cpu().numpy(), Qm.cpu().numpy()
    _assert_bitwise(Qs, Qm, Q0)
    assert np.isfinite(Qs).all()
    assert np.array_equal(s.marker_force(), m.marker_force())


def test_precision_form_and_characteristic_variant(torch_cuda):
    base = W.config2(n=200, h=1.0 / 16.0, sponge=2.0, nprobe=8, rprobe=2.0).with_(n=(160, 150, 1))
    Q0 = W.config2_noisy_state(base)
    for case in (base.with_(precision="mixed32"), base.with_(variables="characteristic", scheme="weno5js")):
        s, m, Qs, Qm, info = _single_and_blocks(torch_cuda, case, Q0, 3, 10)
        _assert_bitwise(Qs, Qm, Q0)


def test_sphere_three_blocks_3d(torch_cuda):
    case = W.config3(n=48, scheme="teno5", nmark=2000)
    Q0 = W.config3_state(case)
    s, m, Qs, Qm, info = _single_and_blocks(torch_cuda, case, Q0, 3, 10)
    _assert_bitwise(Qs, Qm, Q0)
    assert np.array_equal(s.marker_force(), m.marker_force())


def test_block_set_rejections(torch_cuda):
    from paper_1905_00182_amd import fsa

    case = W.config2(n=64, h=1.0 / 16.0, sponge=1.0, nprobe=8, rprobe=1.0)
    with pytest.raises(fsa.FsaError) as e:
        fsa.MultiBlock(case, 17)                 # 64 layers in 17 blocks: thinner than the halo
    assert e.value.code == fsa.EINVAL
    m = fsa.MultiBlock(case, 2)                  # the rotating cylinder's markers
    X = case.markers["X"]
    with pytest.raises(fsa.FsaError) as e:
        m.set_marker_kinematics(X)               # the markers are not EXTERNAL
    assert e.value.code == fsa.ESTATE
    m.set_markers(X, case.markers["dV"], None, "external", 0.0)
    with pytest.raises(fsa.FsaError) as e:
        m.set_marker_kinematics(X + 10.0)        # supports outside the grid
    assert e.value.code == fsa.EINVAL
    with pytest.raises(fsa.FsaError) as e:
        m.set_markers(X + 10.0, case.markers["dV"])  # supports outside the grid
    assert e.value.code == fsa.EINVAL
    # a block's own rejection part-way through (four copies of the markers: more than a block
    # may hold) leaves the markers undefined: the calls that use them refuse until a set succeeds
    dV = case.markers["dV"]
    with pytest.raises(fsa.FsaError) as e:
        m.set_markers(np.concatenate([X] * 4, axis=1), np.concatenate([dV] * 4), None, "external", 0.0)
    assert e.value.code == fsa.EINVAL
    m.scatter(torch_cuda.from_numpy(W.config2_state(case)).cuda())
    for call in (m.marker_force, lambda: m.rk3_steps(case.dt, 1), lambda: m.set_marker_kinematics(X)):
        with pytest.raises(fsa.FsaError) as e:
            call()
        assert e.value.code == fsa.ESTATE
    m.set_markers(X, dV, None, "external", 0.0)
    m.set_marker_kinematics(X)
    m.rk3_steps(case.dt, 1)
    assert np.isfinite(m.marker_force()).all()
