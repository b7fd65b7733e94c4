"""Reference record of the 2048^2 rotating-cylinder case (TENO5, IB, inflow, sponge) from the
CPU oracle only, written to tests/golden/c2_oracle_run.npz.

The run starts from the case's own initial state (the uniform Mach 0.2 stream; the seeded
velocity perturbation enters with the inflow) and takes `--steps` SSP-RK3 steps (4000 by
default: the configured 2000-step run, then as many again so that the cylinder's start-up
wave reaches the radius-50 probe ring).  It records:

  dp_r50[k][360]  Delta p on the configured radius-50 ring after steps 10, 20, ... (every 10)
  dp_r10[k][360]  the same on a radius-10 ring (through step 2000 only)
  force[k][2]     total penalty force on the structure, sum_k F_k dV_k, after the same steps
  norms[m][4], dnorms[m][4]  per-component L2 norm of Q and of Q - Q0 after steps 100, 200, ...
  cells[8192], snap_steps[5], snaps[5][4][8192]  the state at 8192 cells (4096 seeded ones and
                  the 64 x 64 block x in [-1, 3), y in [-2, 2) behind the cylinder) after steps
                  500, 1000, 2000, 3000, 4000

Only oracle/ computes; paper_1905_00182_amd.workloads builds the case and its initial state.
One run takes a few hours on 8 host cores; `--checkpoint DIR` saves the state every 500
steps there and resumes from the latest one.  `--scheme weno5js --steps 200 --out
tests/golden/c2_oracle_run_weno5js_200.npz` writes the companion record of the same set-up in
WENO5-JS, whose continuous weights make the run determined to rounding (a snapshot is also
taken after the last step).
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from paper_1905_00182_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "c2_oracle_run.npz")
EVERY = 10
NORM_EVERY = 100
SNAP_STEPS = (500, 1000, 2000, 3000, 4000)
R10_UNTIL = 2000
SAMPLE_SEED = 20480


def sample_cells(case):
    """8192 distinct cell indices: 4096 seeded uniform ones and a 64 x 64 block behind the
    cylinder."""
    nx, ny = case.n[0], case.n[1]
    i0 = int(round((-1.0 - case.lo[0]) / case.h))
    j0 = int(round((-2.0 - case.lo[1]) / case.h))
    jj, ii = np.meshgrid(np.arange(j0, j0 + 64), np.arange(i0, i0 + 64), indexing="ij")
    block = (jj * nx + ii).ravel()
    rng = np.random.default_rng(SAMPLE_SEED)
    pool = np.setdiff1d(np.arange(nx * ny), block)
    rand = np.sort(rng.choice(pool, size=4096, replace=False))
    return np.concatenate([rand, block]).astype(np.int64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--scheme", default="teno5", choices=["teno5", "weno5js"])
    args = ap.parse_args()

    case = W.config2()
    if args.scheme != case.scheme:
        case = case.with_(scheme=args.scheme)
    nprobe = case.probes.shape[1]
    rings = np.concatenate([case.probes, W.ring_probes(nprobe, 10.0)], axis=1)
    o = Oracle(case.with_(probes=rings))
    Q0 = W.config2_state(case)
    Q = Q0.copy()
    cells = sample_cells(case)
    dV = case.markers["dV"]

    nrec = args.steps // EVERY
    dp_r50 = np.zeros((nrec, nprobe))
    dp_r10 = np.zeros((min(nrec, R10_UNTIL // EVERY), nprobe))
    force = np.zeros((nrec, 2))
    norms = np.zeros((args.steps // NORM_EVERY, case.nq))
    dnorms = np.zeros_like(norms)
    snaps_at = sorted(set([s for s in SNAP_STEPS if s <= args.steps] + [args.steps]))
    snaps = np.zeros((len(snaps_at), case.nq, cells.size))

    start = 0
    ck = None
    if args.checkpoint:
        os.makedirs(args.checkpoint, exist_ok=True)
        ck = os.path.join(args.checkpoint, "c2_oracle_ckpt.npz")
        if os.path.exists(ck):
            z = np.load(ck)
            start = int(z["step"])
            Q = z["Q"].copy()
            o.set_state(z["xi"], float(z["t"]), start)
            dp_r50[: z["dp_r50"].shape[0]] = z["dp_r50"]
            dp_r10[: z["dp_r10"].shape[0]] = z["dp_r10"]
            force[: z["force"].shape[0]] = z["force"]
            norms[: z["norms"].shape[0]] = z["norms"]
            dnorms[: z["dnorms"].shape[0]] = z["dnorms"]
            snaps[: z["snaps"].shape[0]] = z["snaps"]
            print(f"resumed at step {start}", flush=True)

    t0 = time.time()
    for step in range(start + 1, args.steps + 1):
        o.rk3_step(Q, case.dt)
        if step % EVERY == 0:
            k = step // EVERY - 1
            dp = o.probe_dp(Q)
            dp_r50[k] = dp[:nprobe]
            if k < dp_r10.shape[0]:
                dp_r10[k] = dp[nprobe:]
            force[k] = (o.marker_force() * dV).sum(axis=1)
        if step % NORM_EVERY == 0:
            m = step // NORM_EVERY - 1
            for c in range(case.nq):
                norms[m, c] = np.linalg.norm(Q[c])
                dnorms[m, c] = np.linalg.norm(Q[c] - Q0[c])
            print(f"step {step}  {time.time() - t0:.0f} s  max|dp_r50| {np.abs(dp_r50[:k + 1]).max():.3e}",
                  flush=True)
        if step in snaps_at:
            snaps[snaps_at.index(step)] = Q.reshape(case.nq, -1)[:, cells]
        if ck and step % 500 == 0:
            xi, t, st = o.get_state()
            np.savez(ck + ".tmp.npz", step=step, Q=Q, xi=xi, t=t, dp_r50=dp_r50[: step // EVERY],
                     dp_r10=dp_r10[: min(step // EVERY, dp_r10.shape[0])], force=force[: step // EVERY],
                     norms=norms[: step // NORM_EVERY], dnorms=dnorms[: step // NORM_EVERY],
                     snaps=snaps[: sum(1 for s in snaps_at if s <= step)])
            os.replace(ck + ".tmp.npz", ck)

    np.savez_compressed(
        args.out, steps=np.int64(args.steps), every=np.int64(EVERY), norm_every=np.int64(NORM_EVERY),
        dt=np.float64(case.dt), seed=np.int64(case.seed), dp_r50=dp_r50, dp_r10=dp_r10, force=force,
        norms=norms, dnorms=dnorms, cells=cells, snap_steps=np.array(snaps_at, dtype=np.int64), snaps=snaps,
        scheme=np.array(args.scheme), note=np.array("CPU oracle, FP64; see c2_oracle_run.py"))
    print(f"wrote {args.out} after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
