"""The binding rejects device arguments of the wrong dtype, device, layout or shape before any
pointer reaches the library (host-side checks; no GPU needed: the solver object below is
built without a context, and every call must raise before the library is called)."""
import numpy as np
import pytest
import torch

from paper_1905_00182_amd import fsa, workloads as W


def stub_solver(case, nm=8, npr=5):
    s = fsa.Solver.__new__(fsa.Solver)
    s.torch = torch
    s.case = case
    s.dim = case.dim
    s.nq = case.dim + 2
    s.shape = (s.nq,) + case.shape
    s.device = torch.device("cuda", 0)     # a device object only: nothing is allocated on it
    s.ctx = None
    s.workspace = None
    s.nm = nm
    s.np = npr
    return s


CASE = W.config1(n=32)


def meta(shape, dtype=torch.float64):
    # a tensor on the "meta" device has a shape and dtype but no storage
    return torch.empty(shape, dtype=dtype, device="meta")


def test_state_checks():
    s = stub_solver(CASE)
    good_shape = s.shape
    for bad in (torch.zeros(good_shape, dtype=torch.float64),                  # host memory
                meta(good_shape, torch.float32),                              # wrong dtype
                meta((4, 31, 32)),                                            # wrong shape
                np.zeros(good_shape)):                                        # not a tensor
        with pytest.raises(ValueError):
            s.rhs(bad)
        with pytest.raises(ValueError):
            s.rk3_step(bad, 0.01)
        with pytest.raises(ValueError):
            s.probe_dp(bad)
    with pytest.raises(ValueError):                                           # not contiguous
        s._dev(torch.zeros((32, 32, 4), dtype=torch.float64).permute(2, 0, 1), good_shape, torch.float64, "Q")


def test_out_and_field_checks():
    s = stub_solver(CASE)
    cpu = torch.zeros(s.shape, dtype=torch.float64)
    with pytest.raises(ValueError):
        s._dev(cpu, s.shape, torch.float64, "out")
    with pytest.raises(ValueError):
        s.ib_interp(torch.zeros((2, 32, 32), dtype=torch.float32))
    with pytest.raises(ValueError):
        s.ib_interp(torch.zeros((2, 32, 31), dtype=torch.float64))
    with pytest.raises(ValueError):
        s.ib_spread(torch.zeros((2, 7), dtype=torch.float64), torch.zeros((2, 32, 32), dtype=torch.float64))
    with pytest.raises(ValueError):
        s.ib_spread(torch.zeros((2, 8), dtype=torch.float64), torch.zeros((3, 32, 32), dtype=torch.float64))


def test_network_argument_checks():
    s = stub_solver(CASE)
    for bad in (torch.zeros((10, 16), dtype=torch.float64), torch.zeros((10, 15), dtype=torch.float32),
                torch.zeros((10, 16), dtype=torch.float32)):                  # the last: host memory
        with pytest.raises(ValueError):
            s.mlp_forward(bad)
    f = meta((10, 16), torch.float32)
    with pytest.raises(ValueError):
        s._feats(f, meta((9,), torch.uint8))
    with pytest.raises(ValueError):
        s._feats(f, meta((10,), torch.float32))
    # BF16 parameters: bit patterns or a bfloat16 tensor, the network's size
    for bad in (np.zeros(fsa.MLP_NPARAM, dtype=np.float32), np.zeros(fsa.MLP_NPARAM, dtype=np.int64),
                np.zeros(fsa.MLP_NPARAM - 1, dtype=np.uint16), torch.zeros(fsa.MLP_NPARAM, dtype=torch.float32),
                torch.zeros(fsa.MLP_NPARAM + 1, dtype=torch.bfloat16)):
        with pytest.raises(ValueError):
            s.set_mlp_bf16(bad)
