"""TENO5's discrete sub-stencil decisions, GPU against the oracle (Sec. 2: TENO5, with the
sharp cut-off of Fu, Hu & Adams).

The cut-off chi_k < C_T is a discontinuous function of the stencil: where chi_k lies within
rounding of C_T, or where the five values of a stencil differ only by rounding (tails of a
smooth signal that have reached the ambient state's last bits, where chi is a ratio of
rounding noise), two correct FP64 implementations may decide differently.  These tests show
that this is the only place where the library and the oracle differ:

* the library's read-out instantiation (fsa_debug_teno_bits) performs the same arithmetic as
  the production kernels (its step is bit for bit the production step);
* on the same states -- every stage input of the oracle's own runs of the TENO5 cases -- the
  keep pattern the library's stage kernels choose equals the oracle's at every face,
  component and side, except where the library's pattern is the one the oracle itself takes
  on the same five values moved by a few ulps each: a decision within rounding of the
  cut-off, one of several correct results.

The ulps: the split-flux values the two sides reconstruct, f = (F +- alpha q)/2, differ by
a few ulps of their magnitude (the primitives are formed with a Newton-refined reciprocal
instead of a division, products are contracted differently, the wave speeds come from a
different reduction).  A decision counts as a tie when

* the five values spread by at most NOISE_ULPS ulps of their magnitude: the differences the
  indicators are made of then have a few significant bits, as few as the rounding of the
  indicators' own formation (3c - 4d + e of equal values leaves a residue when 3c rounds),
  so the decision is made on rounding noise -- by both sides, differently (with
  epsilon = 1e-40 the cut-off is scale-invariant; exactly uniform regions are such stencils,
  and decide alike at every face, so a free stream stays exact);
* or else the oracle's own TENO5 takes the library's pattern on v + d, with every
  |d_j| <= MAX_ULPS ulps of max|v| (searched over the 3^5 stencils of -1, 0, +1 times
  1, 2, 4, 8 ulps, then seeded random ones): a decision within rounding of the cut-off.
"""
import itertools

import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

from test_gpu_parity_2d import _oracle, _say, _solver

pytestmark = pytest.mark.gpu

MAX_ULPS = 8
NOISE_ULPS = 32


CORNERS = np.array(list(itertools.product((-1.0, 0.0, 1.0), repeat=5)))
RANDOM = np.random.default_rng(1905).uniform(-1.0, 1.0, size=(4000, 5))


def tie_ulps(oracle_mod, v, pattern, ct, max_ulps=MAX_ULPS):
    """Smallest number of ulps (of max|v|: 1, 2, 4, .. max_ulps) by which moving the five
    values lets the oracle's TENO5 choose `pattern`; None if no such move was found."""
    scale = np.spacing(np.abs(v).max())
    moves = np.concatenate([CORNERS, RANDOM])
    u = 1
    while u <= max_ulps:
        if (oracle_mod.teno_flags_n(v + u * scale * moves, ct) == pattern).any():
            return u
        u *= 2
    return None


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def check_decisions(torch, oracle_mod, case, Q0, nsteps, kinematics=None):
    """Run the oracle nsteps from Q0 recording its stage inputs; on each, compare the
    library's keep patterns (a right-hand side with the read-out on) with the oracle's, and
    check every differing one with tie_ulps.  Returns (face-stages compared, differing
    (face, component, side) decisions)."""
    o = _oracle(case)
    o.record_stages(True)
    s = _solver(case)
    bits = s.debug_teno_bits(True)
    Qo = Q0.copy()
    L = torch.empty((case.nq,) + case.shape, dtype=torch.float64, device="cuda")
    compared = mism = nnoise = 0
    ulps = {}
    widest = 0.0
    cache = {}
    shifts = np.array([3 * m + 16 * sd for m in range(case.nq) for sd in (0, 1)])
    for n in range(nsteps):
        t = n * case.dt
        if kinematics is not None:
            o.set_marker_kinematics(*kinematics(case, t))
        o.rk3_step(Qo, case.dt)
        xi_o, t_o, step_o = o.get_state()
        o.set_state(xi_o, t_o, n)        # the inflow ghosts of the step just taken
        for st in range(3):
            X = o.stage_states[st]
            s.set_state(None, t, n)      # (the inflow ghosts' counter; the markers do not
                                         # enter the reconstruction)
            s.rhs(torch.from_numpy(X.copy()).cuda(), out=L)
            gb = bits[0].cpu().numpy().view(np.uint32)
            ob = o.teno_bits(X)
            compared += ob.size
            faces = np.nonzero(gb != ob)[0]
            if faces.size == 0:
                continue
            # every (face, component, side) whose 3-bit pattern differs
            kg = (gb[faces, None].astype(np.int64) >> shifts) & 7
            ko = (ob[faces, None].astype(np.int64) >> shifts) & 7
            fi, ei = np.nonzero(kg != ko)
            g = faces[fi]
            comp, side = shifts[ei] % 16 // 3, shifts[ei] // 16
            V, CHI = o.teno_values(X, g, comp, side)
            pat = kg[fi, ei]
            mism += g.size
            noise = np.ptp(V, axis=1) <= NOISE_ULPS * np.spacing(np.abs(V).max(axis=1))
            nnoise += int(noise.sum())
            for e in np.nonzero(~noise)[0]:
                key = (V[e].tobytes(), int(pat[e]))
                if key not in cache:
                    cache[key] = tie_ulps(oracle_mod, V[e], int(pat[e]), case.teno_ct)
                u = cache[key]
                spread = np.ptp(V[e]) / max(np.abs(V[e]).max(), 1e-300)
                assert u is not None, (
                    f"step {n} stage {st} face {g[e]} comp {comp[e]} side {side[e]}: gpu {pat[e]:03b} oracle "
                    f"{ko[fi[e], ei[e]]:03b}, chi/C_T {CHI[e] / case.teno_ct}, spread {spread:.3e} of the values: "
                    f"the oracle does not take the library's pattern within {MAX_ULPS} ulps of the values")
                ulps[u] = ulps.get(u, 0) + 1
                widest = max(widest, spread)
        o.set_state(xi_o, t_o, step_o)
        _say(f"  step {n}: {mism} differing decisions so far ({nnoise} on noise-flat stencils), all within rounding")
    s.debug_teno_bits(False)
    _say(f"  {case.name} {case.n[:case.dim]}: {compared} face-stages compared, {mism} differing decisions: "
         f"{nnoise} on stencils flat to {NOISE_ULPS} ulps, the others the oracle's own within rounding (ulps "
         f"needed: {dict(sorted(ulps.items()))}; widest relative spread {widest:.2e})")
    return compared, mism


def test_readout_instantiation_is_the_production_arithmetic(torch_cuda):
    torch = torch_cuda
    for case, Q0 in ((W.config2(n=160, nprobe=8, rprobe=3.0, sponge=1.0), None),
                     (W.config3(n=64, scheme="teno5", nmark=1000), None)):   # (n_x = 64: the last x face column too)
        Q0 = W.config2_noisy_state(case) if case.dim == 2 else W.config3_state(case)
        out = []
        for dbg in (False, True):
            s = _solver(case)
            if dbg:
                bits = s.debug_teno_bits(True)
            Q = torch.from_numpy(Q0.copy()).cuda()
            s.rk3_steps(Q, case.dt, 2)
            s.sync()
            out.append(Q.cpu().numpy())
            if dbg:
                b = bits.cpu().numpy()
                assert (b != 0).all()          # every face of every stage was written
            s.close()
        assert np.array_equal(out[0], out[1]), case.name


def test_readout_rejects_other_forms(torch_cuda):
    from paper_1905_00182_amd import fsa

    for case in (W.config1(n=64), W.config2(n=64, nprobe=8, rprobe=1.0, sponge=1.0).with_(precision="mixed32")):
        s = _solver(case)
        with pytest.raises(fsa.FsaError) as e:
            s.debug_teno_bits(True)
        assert e.value.code == fsa.EUNSUPPORTED


def test_decisions_config3_pulse(torch_cuda, oracle_mod):
    case = W.config3(n=48, scheme="teno5", nmark=2000)
    check_decisions(torch_cuda, oracle_mod, case, W.config3_state(case), 30)


def test_decisions_config2_uniform_start(torch_cuda, oracle_mod):
    case = W.config2(n=256, nprobe=16, rprobe=4.0, sponge=2.0)
    check_decisions(torch_cuda, oracle_mod, case, W.config2_state(case), 20)


def test_decisions_flapping_plate(torch_cuda, oracle_mod):
    case = W.config5(n=128, L=8.0, nmark=128, scheme="teno5")
    check_decisions(torch_cuda, oracle_mod, case, W.uniform_state(case), 20, kinematics=W.plate_kinematics)


def test_decisions_hovering_insect(torch_cuda, oracle_mod):
    case = W.insect(n=192, L=3.84, sponge=0.5, nprobe=16, rprobe=1.5)
    check_decisions(torch_cuda, oracle_mod, case, W.uniform_state(case), 20, kinematics=W.insect_kinematics)
