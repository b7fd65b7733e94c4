"""The oracle's test hooks on TENO5 decisions (stage-state recording, per-face keep patterns,
per-face chi) against the oracle's own definitions: they add nothing to what it computes."""
import numpy as np
import pytest

from paper_1905_00182_amd import workloads as W

CT = 1e-6



@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_state_decides_alike_everywhere(oracle_mod, dim):
    # every face of a direction sees the same five values, so the same decisions.  (Not
    # necessarily all kept: for a value v whose 3v rounds, t2 = 3c - 4d + e leaves a rounding
    # residue, and with epsilon = 1e-40 TENO5 then cuts on that noise -- identically at every
    # face, so the free stream stays exact.)
    case = W.periodic_box(dim=dim, n=12, scheme="teno5", prim_inf=(1.0, 0.3, -0.1, 0.2, 1.0 / W.GAMMA))
    o = oracle_mod.Oracle(case)
    b = o.teno_bits(W.uniform_state(case))
    assert b.size == sum(o.face_counts()) == dim * 13 * 12 ** (dim - 1)
    off = 0
    for n in o.face_counts():
        assert (b[off:off + n] == b[off]).all()
        off += n


@pytest.mark.parametrize("dim", [2, 3])
def test_face_bits_follow_chi(oracle_mod, dim):
    # every recorded decision is chi_k >= C_T on the detail's values, which are the split
    # fluxes the right-hand side reconstructs; a jump makes cut-offs
    n = (20, 16, 12) if dim == 3 else (24, 20)
    case = W.periodic_box(dim=dim, n=n[0], scheme="teno5").with_(n=tuple(n) + (1,) * (3 - dim))
    Q = W.perturbed_state(case, seed=3, amp=2e-2, step_amp=0.3)
    o = oracle_mod.Oracle(case)
    b = o.teno_bits(Q)
    rng = np.random.default_rng(4)
    cut = 0
    lins = rng.choice(b.size, size=300, replace=False)
    g = np.repeat(lins, 2 * case.nq)
    m = np.tile(np.repeat(np.arange(case.nq), 2), lins.size)
    sd = np.tile([0, 1], lins.size * case.nq)
    V, CHI = o.teno_values(Q, g, m, sd)
    got = oracle_mod.teno_flags_n(V)
    for e in range(g.size):
        want = sum(1 << k for k in range(3) if not CHI[e, k] < CT)
        assert (int(b[g[e]]) >> (3 * m[e] + 16 * sd[e])) & 7 == want == got[e]
        assert want == oracle_mod.teno_flags(V[e])
        cut += want != 7
    assert cut > 0


def test_recorded_stage_states(oracle_mod):
    case = W.periodic_box(dim=2, n=24, scheme="teno5", mu=0.003)
    Q0 = W.perturbed_state(case, seed=5, amp=1e-2, step_amp=0.2)
    o = oracle_mod.Oracle(case)
    o.record_stages(True)
    Q = o.rk3_step(Q0.copy(), case.dt)
    S = o.stage_states
    dt = case.dt
    assert np.array_equal(S[0], Q0)
    ref = oracle_mod.Oracle(case)
    Q1 = Q0 + dt * ref.rhs(Q0)
    assert np.array_equal(S[1], Q1)
    Q2 = 0.75 * Q0 + 0.25 * (Q1 + dt * ref.rhs(Q1))
    assert np.array_equal(S[2], Q2)
    assert np.array_equal(Q, (1.0 / 3.0) * Q0 + (2.0 / 3.0) * (Q2 + dt * ref.rhs(Q2)))
    o.record_stages(False)
    o.rk3_step(Q.copy(), dt)            # recording off: the buffer is left as it was
    assert np.array_equal(o.stage_states[0], Q0)
