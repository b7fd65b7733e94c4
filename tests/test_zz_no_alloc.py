"""fsa_alpha_noalloc (no context, partials in the library's static device scratch) against
fsa_alpha (a context's workspace) on the same states: two calls in a row, the second on a
smaller grid, bit for bit (a maximum does not depend on the order of its operands)."""
import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fsa_mod():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1905_00182_amd import fsa

    fsa.lib()
    return fsa


def with_context(fsa_mod, case, Q):
    s = fsa_mod.Solver(case.with_(markers=None, probes=None))
    a = s.alpha(Q)
    s.close()
    return a


def test_noalloc_alpha_matches_the_context_entry_point(fsa_mod):
    import torch

    # a grid with more cells than 2048 blocks of 256 (folded into the same partials), then a
    # smaller 2D grid, then a 3D one: each against the context entry point on the same state
    big = W.periodic_box(dim=2, n=1024).with_(n=(1024, 600, 1))
    small = W.periodic_box(dim=2, n=96).with_(n=(96, 80, 1))
    cube = W.periodic_box(dim=3, n=24).with_(n=(24, 20, 18))
    out = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
    for k, case in enumerate((big, small, cube)):
        Q0 = W.perturbed_state(case.with_(prim_inf=(1.0, 0.3, -0.2, 0.1, 1.0 / W.GAMMA)), seed=11 + k, amp=0.05)
        Q = torch.from_numpy(Q0).cuda()
        fsa_mod.alpha_noalloc(case, Q, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want = with_context(fsa_mod, case, Q)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (case.n, got, want)
        assert got[: case.dim].min() > 1.0 and (case.dim == 3 or got[2] == 0.0)


def test_noalloc_alpha_propagates_nan_and_rejects_bad_arguments(fsa_mod):
    import torch

    case = W.periodic_box(dim=2, n=64)
    Q = torch.from_numpy(W.uniform_state(case)).cuda()
    Q[0, 10, 10] = float("nan")
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    fsa_mod.alpha_noalloc(case, Q, out)
    torch.cuda.synchronize()
    assert np.isnan(out[0].item()) and np.isnan(out[1].item())
    with pytest.raises(ValueError):
        fsa_mod.alpha_noalloc(case, Q, torch.zeros(2, dtype=torch.float64, device="cuda"))
    bad = fsa_mod.make_desc(case)
    bad.dim = 5
    rc = fsa_mod.lib().fsa_alpha_noalloc(fsa_mod.C.byref(bad), fsa_mod._ptr(Q), fsa_mod._ptr(out), None)
    assert rc == fsa_mod.EINVAL
