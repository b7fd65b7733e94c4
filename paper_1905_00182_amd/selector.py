"""Training of the learned TENO5 sub-stencil selector on the GPU.

Every arithmetic step runs in the library's kernels (harvest, BF16 MFMA forward/backward,
Adam); this module only orders the calls: it runs short FP64 trajectories, harvests their
significant face sides with their FP64 TENO5 labels, shuffles them and takes Adam steps on
mini-batches.
"""
import numpy as np

from . import fsa
from . import workloads as W

NPARAM = fsa.MLP_NPARAM
_SHAPES = [(15, 32), (32,), (32, 32), (32,), (32, 3), (3,)]


def init_params(seed):
    """He initialisation (weights ~ N(0, 2 / fan_in), biases 0), flat FP32 [1667]."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp in _SHAPES:
        if len(shp) == 2:
            parts.append(rng.normal(0.0, np.sqrt(2.0 / shp[0]), size=shp).reshape(-1))
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts).astype(np.float32)


def training_cases(n1=128, n2=2048, n3=128, n5=512, every2=200):
    """FP64 runs whose face sides train the selector (about 1e7 sides): the cylinder
    scattering case with TENO5 (config 1), the rotating-cylinder case at its full size from
    its uniform start (config 2, a state every `every2` steps: the start-up wave, wake and
    inflow noise), the sphere-scattering case in 3D (config 3's set-up at n3^3, its sides in
    all three directions) and the rigid flapping plate (config 5's cell size, the wake inside
    [-2, 2]^2, a tenth of its sides without a cut-off kept so that its mostly smooth wake does
    not crowd out the rest), each with its initial state, sampling interval and the keep rate
    of its all-kept sides (every side with a cut-off is kept)."""
    c1 = W.config1(n=n1, scheme="teno5")
    c2 = W.config2(n=n2, nprobe=8, rprobe=3.0)
    c3 = W.config3(n=n3, scheme="teno5", nmark=2000)
    c5 = W.config5(n=n5, L=n5 / 64.0)
    return [(c1, W.config1_state(c1), 20), (c2, W.config2_state(c2), every2), (c3, W.config3_state(c3), 40),
            (c5, W.uniform_state(c5), 300, 0.1)]


def harvest(cases, chunks=6, keep_rate=1.0, seed=100, cap=1 << 22):
    """Significant face sides (features [n, 16] FP32, labels [n] uint8) from the states of FP64
    runs of each case, sampled every `every` steps (chunks + 1 states per case); a case with
    plate kinematics has its markers moved before every step.  A case may carry its own keep
    rate of the sides without a cut-off (fourth tuple entry; every cut-off side is kept)."""
    import torch

    F, L = [], []
    for item in cases:
        case, Q0, every = item[:3]
        rate = item[3] if len(item) > 3 else keep_rate
        s = fsa.Solver(case.with_(precision="fp64"))
        Q = torch.from_numpy(np.ascontiguousarray(Q0)).cuda()
        moving = "plate" in case.extra     # markers moved before every step
        n = 0
        for k in range(chunks + 1):
            if k and moving:
                for _ in range(every):
                    s.set_marker_kinematics(*W.plate_kinematics(case, n * case.dt))
                    if n:
                        s.rk3_steps_resume(Q, case.dt)
                    else:
                        s.rk3_step(Q, case.dt)
                    n += 1
            elif k:
                s.rk3_steps(Q, case.dt, every)
            f, lab, _ = s.harvest(Q, rate, seed + k, cap)
            F.append(f.clone())
            L.append(lab.clone())
        s.sync()
        s.close()
    return torch.cat(F), torch.cat(L)


def train(F, L, steps=4000, batch=4096, lr=3e-3, lr_final=1e-3, final_frac=0.25, seed=42, conf=0.8,
          report_every=500):
    """Adam on shuffled mini-batches; returns (parameters [1667] FP32, sampled losses)."""
    import torch

    tr = fsa.Solver(W.config2(n=64, h=1.0 / 16.0, sponge=1.0, nprobe=0).with_(precision="learned32"))
    tr.mlp_set(init_params(seed), conf)
    g = torch.Generator().manual_seed(seed)
    perm = torch.randperm(F.shape[0], generator=g).to(F.device)
    F, L = F[perm].contiguous(), L[perm].contiguous()
    loss = torch.empty(1, dtype=torch.float32, device=F.device)
    nb = max(F.shape[0] // batch, 1)
    losses = []
    for step in range(steps):
        a = (step % nb) * batch
        rate = lr if step < (1.0 - final_frac) * steps else lr_final
        tr.mlp_train_step(F[a:a + batch], L[a:a + batch], rate, loss)
        if step % report_every == 0 or step == steps - 1:
            losses.append(float(loss.item()))
    theta = tr.mlp_get()
    tr.close()
    return theta, losses
