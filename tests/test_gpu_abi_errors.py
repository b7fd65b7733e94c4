"""Error behaviour of the C ABI as declared in include/fsa.h: invalid descriptors, arguments and
call orders return their status codes (raised by the binding as FsaError) and leave the
context usable."""
import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fsa_mod():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1905_00182_amd import fsa

    return fsa


def _box(dim=2, n=24, **kw):
    c = W.periodic_box(dim=dim, n=n, scheme="teno5", mu=0.003)
    return c.with_(**kw) if kw else c


@pytest.mark.parametrize("change, code", [
    ({"gamma": 1.0}, "EINVAL"),
    ({"mu": -1.0}, "EINVAL"),
    ({"bc": (("periodic", "extrap"), ("periodic", "periodic"), ("periodic", "periodic"))}, "EINVAL"),
    ({"sponge_width": ((-1.0, 0.0), (0.0, 0.0), (0.0, 0.0))}, "EINVAL"),
    ({"prim_inf": (0.0, 0.0, 0.0, 0.0, 1.0)}, "EINVAL"),
    ({"extra": {"selector_stride": 2}}, "EINVAL"),
])
def test_invalid_descriptor(fsa_mod, change, code):
    with pytest.raises(fsa_mod.FsaError) as e:
        fsa_mod.Solver(_box(**change))
    assert e.value.code == getattr(fsa_mod, code)


def test_learned_form_in_3d_unsupported(fsa_mod):
    with pytest.raises(fsa_mod.FsaError) as e:
        fsa_mod.Solver(_box(dim=3, n=12, precision="learned32"))
    assert e.value.code == fsa_mod.EUNSUPPORTED


def test_argument_and_order_errors(fsa_mod):
    import torch

    case = _box()
    s = fsa_mod.Solver(case)
    Q = torch.from_numpy(W.perturbed_state(case, seed=1, amp=1e-2)).cuda()
    lib = fsa_mod.lib()
    p = fsa_mod._ptr(Q)
    assert lib.fsa_rhs(s.ctx, p, p) == fsa_mod.EINVAL                    # output aliases input
    assert lib.fsa_rk3_steps(s.ctx, p, 0.0, 1) == fsa_mod.EINVAL          # dt must be positive
    assert lib.fsa_rk3_steps(s.ctx, p, case.dt, 0) == fsa_mod.EINVAL      # nsteps must be positive
    assert lib.fsa_diagnostics(s.ctx, p, None, None) == fsa_mod.EINVAL    # nothing requested
    assert lib.fsa_mlp_get(s.ctx, np.zeros(fsa_mod.MLP_NPARAM, np.float32).ctypes.data,
                           fsa_mod.MLP_NPARAM) == fsa_mod.ESTATE          # no network yet
    with pytest.raises(fsa_mod.FsaError) as e:
        s.mlp_set(np.zeros(fsa_mod.MLP_NPARAM), conf_threshold=1.5)
    assert e.value.code == fsa_mod.EINVAL
    # the context still works after the rejected calls
    L = s.rhs(Q)
    s.sync()
    assert torch.isfinite(L).all()


def test_resume_needs_the_state_of_the_last_step_call(fsa_mod):
    import torch

    case = _box()
    s = fsa_mod.Solver(case)
    Q = torch.from_numpy(W.perturbed_state(case, seed=2, amp=1e-2)).cuda()
    Q2 = Q.clone()
    lib = fsa_mod.lib()
    p, p2 = fsa_mod._ptr(Q), fsa_mod._ptr(Q2)
    assert lib.fsa_rk3_steps_resume(s.ctx, p, case.dt, 1) == fsa_mod.ESTATE    # no step call yet
    s.rk3_step(Q, case.dt)
    assert lib.fsa_rk3_steps_resume(s.ctx, p2, case.dt, 1) == fsa_mod.ESTATE   # another buffer
    assert lib.fsa_rk3_steps_resume(s.ctx, p, 0.0, 1) == fsa_mod.EINVAL        # dt must be positive
    s.rk3_steps_resume(Q, case.dt)                                               # the state it left
    s.rk3_steps_resume(Q, case.dt, 2)
    s.rhs(Q2)
    assert lib.fsa_rk3_steps_resume(s.ctx, p, case.dt, 1) == fsa_mod.ESTATE    # slot reused since
    s.rk3_step(Q, case.dt)
    s.rk3_steps_resume(Q, case.dt)
    s.sync()
    assert torch.isfinite(Q).all()


def test_learned_form_needs_a_network(fsa_mod):
    import torch

    case = _box(precision="learned32")
    s = fsa_mod.Solver(case)
    Q = torch.from_numpy(W.uniform_state(case)).cuda()
    with pytest.raises(fsa_mod.FsaError) as e:
        s.rk3_step(Q, case.dt)
    assert e.value.code == fsa_mod.ESTATE


def test_harvest_rejections_and_a_uniform_3d_state(fsa_mod):
    """A keep rate outside [0, 1] is refused; a uniform 3D state has no significant side."""
    import torch

    case = _box(dim=3, n=12)
    s = fsa_mod.Solver(case)
    Q = torch.from_numpy(W.uniform_state(case)).cuda()
    for rate in (-0.5, 1.5, float("nan")):
        with pytest.raises(fsa_mod.FsaError) as e:
            s.harvest(Q, rate, 1, 16)
        assert e.value.code == fsa_mod.EINVAL
    feats, labels, n = s.harvest(Q, 1.0, 1, 16)
    assert n == 0 and feats.shape[0] == 0


def test_coupled_steps_need_the_plates_markers(fsa_mod):
    import torch

    case = W.config5_flexible(n=128, L=8.0, nmark=128, nel=10)
    plate = fsa_mod.Plate(case)
    Q = torch.from_numpy(W.uniform_state(case)).cuda()
    n, motion, dim = fsa_mod.C.c_int32(), fsa_mod.C.c_int32(), fsa_mod.C.c_int32()
    s = fsa_mod.Solver(case)
    assert fsa_mod.lib().fsa_marker_info(s.ctx, fsa_mod.C.byref(n), fsa_mod.C.byref(motion),
                                         fsa_mod.C.byref(dim)) == fsa_mod.OK
    assert (n.value, motion.value, dim.value) == (128, fsa_mod.MOTION["external"], 2)
    for other in (W.config5_flexible(n=128, L=8.0, nmark=96, nel=10),          # fewer markers
                  case.with_(markers={**case.markers, "motion": "static"})):  # not EXTERNAL
        so = fsa_mod.Solver(other)
        with pytest.raises(fsa_mod.FsaError) as e:
            plate.coupled_steps(so, Q, case.dt, 1, resume=False)
        assert e.value.code == fsa_mod.ESTATE
        so.close()
    # a 3D solver with as many EXTERNAL markers: its [3][n] arrays are not the plate's [2][n]
    c3 = W.config3(n=16, nmark=128, L=4.0)
    X3 = np.stack([np.linspace(-0.5, 0.5, 128), np.zeros(128), np.zeros(128)])
    c3 = c3.with_(markers={"X": X3, "dV": np.full(128, 1.0 / 128), "U": None, "motion": "external", "omega": 0.0})
    s3 = fsa_mod.Solver(c3)
    Q3 = torch.from_numpy(W.uniform_state(c3)).cuda()
    with pytest.raises(fsa_mod.FsaError) as e:
        plate.coupled_steps(s3, Q3, c3.dt, 1, resume=False)
    assert e.value.code == fsa_mod.EUNSUPPORTED
    s3.close()
    plate.coupled_steps(s, Q, case.dt, 2, resume=False)      # the matching pair still works
    s.sync()
    assert torch.isfinite(Q).all()


def test_binding_rejects_wrong_shapes(fsa_mod):
    case = W.config5(n=128, L=8.0, nmark=64)
    s = fsa_mod.Solver(case)
    X, U = W.plate_kinematics(case, 0.0)
    for bad in (X[:, :-1], X.T, X[:1]):
        with pytest.raises(ValueError):
            s.set_marker_kinematics(bad, U)
    with pytest.raises(ValueError):
        s.set_probes(np.zeros((3, 4)))
    with pytest.raises(ValueError):
        s.set_state(np.zeros((2, 63)), 0.0, 0)
    s.set_marker_kinematics(X, U)    # the right shapes still work
    s.sync()


def test_workspace_capacities_are_enforced(fsa_mod):
    import torch

    case = W.config1(n=64)
    s = fsa_mod.Solver(case.with_(extra={"max_markers": 64, "max_probes": 32}))
    need = fsa_mod.C.c_size_t()
    assert fsa_mod.lib().fsa_workspace_bytes(fsa_mod.C.byref(s.desc), fsa_mod.C.byref(need)) == fsa_mod.OK
    assert s.workspace.numel() == need.value and s.workspace.is_cuda
    X, dV = W.circle_markers(65, 0.5)
    with pytest.raises(fsa_mod.FsaError) as e:
        s.set_markers(X, dV)                                     # one more than the capacity
    assert e.value.code == fsa_mod.EINVAL and "max_markers" in str(e.value)
    with pytest.raises(fsa_mod.FsaError) as e:
        s.set_probes(W.ring_probes(33, 2.0))
    assert e.value.code == fsa_mod.EINVAL
    # a window capacity that the markers' supports outgrow
    sw = fsa_mod.Solver(case.with_(markers=None, extra={"max_markers": 64, "max_window_cells": 40}))
    X, dV = W.circle_markers(64, 0.5)
    with pytest.raises(fsa_mod.FsaError) as e:
        sw.set_markers(X, dV)
    assert e.value.code == fsa_mod.EINVAL and "max_window_cells" in str(e.value)
    # within the capacities the context still steps
    s.set_markers(*W.circle_markers(64, 0.5))
    Q = torch.from_numpy(W.config1_state(case)).cuda()
    s.rk3_step(Q, case.dt)
    s.sync()
    assert torch.isfinite(Q).all()
    s.close()
    sw.close()
