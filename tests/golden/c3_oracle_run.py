"""Reference record of the 256^3 sphere-scattering case (config 3's set-up: quiescent gas, the
Gaussian pulse at (2, 0, 0), the sphere of 10^4 markers, sponge) from the CPU oracle only,
written to tests/golden/c3_oracle_run_<scheme>.npz.

The run takes the case's configured 500 SSP-RK3 steps from its initial state in WENO5-JS by
default, whose continuous weights leave the run determined to rounding, so that a second
implementation can be held to rounding over the whole run.  It records:

  dp[k][64]       Delta p on the case's 64 probes (radius 4) after steps 5, 10, ... (every 5)
  force[k][3]     total penalty force on the sphere, sum_k F_k dV_k, after the same steps
  norms[m][5], dnorms[m][5]  per-component L2 norm of Q and of Q - Q0 after steps 50, 100, ...
  cells[8192], snap_steps, snaps[s][5][8192]  the state at 8192 cells (4096 seeded ones and
                  the 16 x 16 x 16 block around the pulse's start) after steps 100, 250, 500

Only oracle/ computes; paper_1905_00182_amd.workloads builds the case and its initial state.
One run takes about three hours on 8 host cores; `--checkpoint DIR` saves the state every 50
steps there and resumes from the latest one.
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

EVERY = 5
NORM_EVERY = 50
SNAP_STEPS = (100, 250, 500)
SAMPLE_SEED = 25600


def sample_cells(case):
    """8192 distinct cell indices: 4096 seeded uniform ones and the 16^3 block around the
    pulse's start."""
    nx, ny, nz = case.n
    c = [int(round((x - case.lo[d]) / case.h)) for d, x in enumerate((2.0, 0.0, 0.0))]
    kk, jj, ii = np.meshgrid(np.arange(c[2] - 8, c[2] + 8), np.arange(c[1] - 8, c[1] + 8),
                             np.arange(c[0] - 8, c[0] + 8), indexing="ij")
    block = ((kk * ny + jj) * nx + ii).ravel()
    rng = np.random.default_rng(SAMPLE_SEED)
    pool = np.setdiff1d(np.arange(nx * ny * nz), block)
    rand = np.sort(rng.choice(pool, size=4096, replace=False))
    return np.concatenate([rand, block]).astype(np.int64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scheme", default="weno5js", choices=["teno5", "weno5js"])
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    out = args.out or os.path.join(HERE, f"c3_oracle_run_{args.scheme}.npz")

    case = W.config3(n=256, scheme=args.scheme)
    o = Oracle(case)
    Q0 = W.config3_state(case)
    Q = Q0.copy()
    cells = sample_cells(case)
    dV = case.markers["dV"]
    npr = case.probes.shape[1]
    nrec = args.steps // EVERY
    dp = np.zeros((nrec, npr))
    force = np.zeros((nrec, 3))
    norms = np.zeros((args.steps // NORM_EVERY, case.nq))
    dnorms = np.zeros_like(norms)
    snaps_at = sorted(set([s for s in SNAP_STEPS if s <= args.steps] + [args.steps]))
    snaps = np.zeros((len(snaps_at), case.nq, cells.size))

    start = 0
    ck = None
    if args.checkpoint:
        os.makedirs(args.checkpoint, exist_ok=True)
        ck = os.path.join(args.checkpoint, f"c3_oracle_ckpt_{args.scheme}.npz")
        if os.path.exists(ck):
            z = np.load(ck)
            start = int(z["step"])
            Q = z["Q"].copy()
            o.set_state(z["xi"], float(z["t"]), start)
            for name, arr in (("dp", dp), ("force", force), ("norms", norms), ("dnorms", dnorms), ("snaps", snaps)):
                arr[: z[name].shape[0]] = z[name]
            print(f"resumed at step {start}", flush=True)

    t0 = time.time()
    for step in range(start + 1, args.steps + 1):
        o.rk3_step(Q, case.dt)
        if step % EVERY == 0:
            k = step // EVERY - 1
            dp[k] = o.probe_dp(Q)
            force[k] = (o.marker_force() * dV).sum(axis=1)
        if step % NORM_EVERY == 0:
            m = step // NORM_EVERY - 1
            for c in range(case.nq):
                norms[m, c] = np.linalg.norm(Q[c])
                dnorms[m, c] = np.linalg.norm(Q[c] - Q0[c])
            print(f"step {step}  {time.time() - t0:.0f} s  max|dp| {np.abs(dp[:k + 1]).max():.3e}", flush=True)
        if step in snaps_at:
            snaps[snaps_at.index(step)] = Q.reshape(case.nq, -1)[:, cells]
        if ck and step % NORM_EVERY == 0:
            xi, t, st = o.get_state()
            np.savez(ck + ".tmp.npz", step=step, Q=Q, xi=xi, t=t, dp=dp[: step // EVERY],
                     force=force[: step // EVERY], norms=norms[: step // NORM_EVERY],
                     dnorms=dnorms[: step // NORM_EVERY], snaps=snaps[: sum(1 for s in snaps_at if s <= step)])
            os.replace(ck + ".tmp.npz", ck)

    np.savez_compressed(
        out, steps=np.int64(args.steps), every=np.int64(EVERY), norm_every=np.int64(NORM_EVERY),
        dt=np.float64(case.dt), scheme=np.array(args.scheme), dp=dp, force=force, norms=norms, dnorms=dnorms,
        cells=cells, snap_steps=np.array(snaps_at, dtype=np.int64), snaps=snaps,
        note=np.array("CPU oracle, FP64; see c3_oracle_run.py"))
    print(f"wrote {out} after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
