"""Benchmark: SSP-RK3 steps of the 2048^2 TENO5 rotating-cylinder case on one MI355X.

A step is one pass of the whole hot path: for each of the three stages, the global
Lax-Friedrichs wave-speed reduction, the penalty immersed-boundary step (interpolation,
feedback force, spreading) and the fused stencil/update kernel (flux splitting, TENO5
reconstruction in x and y, fourth-order viscous terms, IB and sponge sources, RK3 update).
Inputs are synthetic (the uniform Mach 0.2 stream; the seeded perturbation enters with the
inflow) and resident in HBM before the timed region.

Variants (unless --no-variants): the whole run of the same case (the configured 2000 steps
and their continuation to 4000, by which the cylinder's start-up wave crosses the radius-50
ring) in FP64, in the FP32 precision form and in the FP32 + learned-selector form (network
trained first, in process, by the library's own kernels from FP64 runs of configs 1-3 and the
plate), each timed over the run with the acoustic pressure sampled every 10 steps on the 360
probes of the radius-50 ring and on a radius-10 ring; each form's probe signal is compared
with the CPU oracle's record of the same run (tests/golden/c2_oracle_run.npz, when present)
and with the FP64 GPU run.  The learned form is also run with the selector evaluated once
per step.

Prints one JSON line.  Metric: cell-stage updates per second (cells x 3 stages x steps /
wall time).  roofline: the fused stage kernel, whose launches are bracketed by HIP events on
the library's stream inside the timed region; its algorithmic FP64 operation count per
cell-stage is stated in ALGO_FLOPS below.  cpu_baseline: the FP64 CPU oracle on a few steps
of the same case on this host's cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector peak (256 CU x 2.4 GHz x 128 flop/clk)
PEAK_HBM_GBPS = 8000.0
# Algorithmic FP64 operations per cell-stage of the 2D path (one op = one add, mul, div,
# sqrt or compare of the method's plain formulation; see the design notes for the count).
ALGO_FLOPS_2D = {"teno5": 1591, "weno5js": 1303}
ALGO_BYTES_2D = 256.0 / 3.0  # FP64 state: read Qs (+ Qn in stages 2-3), write Q_{s+1}
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_stage2d_teno5_2048_pmc.txt")
KERNEL_SOURCES = ["paper_1905_00182_amd/csrc/k_stage2d.hip", "paper_1905_00182_amd/csrc/fsa_dev.hpp"]


_T0 = time.perf_counter()


def progress(msg):
    """A progress line on stderr (the JSON result is the one line on stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(launch_cells):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, or None when the
    summary is missing or was taken on a different kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    vals = {}
    for line in open(PMC_SUMMARY):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(case, steps, steps_1t=1):
    """The FP64 CPU oracle on this host: `steps` SSP-RK3 steps of the case with every core's
    OpenMP thread, then `steps_1t` with one thread (each after a warm-up step)."""
    from oracle import oracle as ora
    from paper_1905_00182_amd import workloads as W

    Q = W.config2_state(case)
    o = ora.Oracle(case)
    threads = ora.threads()
    o.rk3_step(Q, case.dt)            # warm-up step (page-in, thread start)
    t0 = time.perf_counter()
    for _ in range(steps):
        o.rk3_step(Q, case.dt)
    dt = time.perf_counter() - t0
    one = None
    if steps_1t > 0:
        ora.threads(1)
        o.rk3_step(Q, case.dt)
        t1 = time.perf_counter()
        for _ in range(steps_1t):
            o.rk3_step(Q, case.dt)
        dt1 = time.perf_counter() - t1
        ora.threads(threads)
        one = {"value": round(case.ncell * 3 * steps_1t / dt1 / 1e6, 3), "cores": 1,
               "sample": f"{steps_1t} step(s) after one warm-up step ({dt1:.1f} s)"}
    return {
        "value": case.ncell * 3 * steps / dt / 1e6,
        "unit": "Mcell-stage/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": f"{steps} SSP-RK3 steps of the same {case.n[0]}x{case.n[1]} case after one warm-up step "
                  f"({dt:.1f} s, FP64 C oracle, OpenMP)",
        "one_thread": one,
    }


def full_run(case, Q0, nsteps, every, net=None):
    """nsteps SSP-RK3 steps from Q0 with the probe pressure sampled every `every` steps;
    returns wall seconds, probe samples [nsteps / every][probes] and the final stats.  The
    solver is warmed up (tuning launch, page-in) on a copy first and reset to step 0."""
    import numpy as np
    import torch

    from paper_1905_00182_amd import fsa

    s = fsa.Solver(case)
    if net is not None:
        s.mlp_set(net, 0.8)
    Qw = Q0.clone()
    s.rk3_steps(Qw, case.dt, 2)
    s.sync()
    s.set_state(np.zeros((case.dim, s.nm)), 0.0, 0)
    stats0 = s.stats()
    Q = Q0.clone()
    nsamp = nsteps // every
    dps = torch.empty((nsamp, s.np), dtype=torch.float64, device=Q.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nsamp):
        s.rk3_steps(Q, case.dt, every) if k == 0 else s.rk3_steps_resume(Q, case.dt, every)
        s.probe_dp(Q, out=dps[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = s.stats()
    s.close()
    sides = st.learned_sides - stats0.learned_sides
    return wall, dps, {
        "significant": (st.significant_sides - stats0.significant_sides) / sides if sides else None,
        "fallback": (st.fallback_sides - stats0.fallback_sides) / sides if sides else None,
    }


ORACLE_RECORD = os.path.join(ROOT, "tests", "golden", "c2_oracle_run.npz")


def variants(case, Q0, nsteps, every=10, plate_steps=None):
    """The FP64, precision and learned forms over the whole run (probes on the configured
    radius-50 ring and a radius-10 ring, sampled every `every` steps), each form's acoustic
    error against the CPU oracle's record of the same run (tests/golden/c2_oracle_run.npz,
    written by the oracle alone) and against the FP64 GPU run."""
    import numpy as np
    import torch

    from paper_1905_00182_amd import selector
    from paper_1905_00182_amd import workloads as W

    t0 = time.perf_counter()
    F, L = selector.harvest(selector.training_cases())
    net, losses = selector.train(F, L)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    progress(f"selector trained on {F.shape[0]} sides in {t_train:.1f} s")
    nprobe = case.probes.shape[1]
    rings = case.with_(probes=np.concatenate([case.probes, W.ring_probes(nprobe, 10.0)], axis=1))
    rec = None
    if os.path.exists(ORACLE_RECORD):
        z = np.load(ORACLE_RECORD)
        if int(z["every"]) == every and abs(float(z["dt"]) - case.dt) == 0.0:
            rec = {"r50": torch.from_numpy(z["dp_r50"]).cuda(), "r10": torch.from_numpy(z["dp_r10"]).cuda()}
    res = {}
    cs = case.ncell * 3 * nsteps
    runs = {}
    forms = (("fp64", "fp64", None, 1, "component"), ("mixed32", "mixed32", None, 1, "component"),
             ("learned32", "learned32", net, 1, "component"), ("learned32_stride3", "learned32", net, 3, "component"),
             ("fp64_characteristic", "fp64", None, 1, "characteristic"))
    for name, prec, n, stride, var in forms:
        runs[name] = full_run(rings.with_(precision=prec, variables=var, extra={"selector_stride": stride}), Q0,
                              nsteps, every, n)
        progress(f"C2 {name}: {nsteps} steps in {runs[name][0]:.2f} s")

    def err(a, b):
        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))

    w64, dp64, _ = runs["fp64"]
    for name, (w, dp, fr) in runs.items():
        e = {"value": round(cs / w / 1e6, 3), "ms_per_step": round(w / nsteps * 1e3, 4)}
        if name == "fp64_characteristic":
            # another reconstruction of the method, not an approximation of the FP64 run: its
            # acoustic pressure differs from the component-wise one by the schemes' difference
            e["speedup_vs_fp64"] = round(w64 / w, 3)
            e["acoustic_diff_r50_vs_component"] = err(dp[:, :nprobe], dp64[:, :nprobe])
            e["acoustic_diff_r10_vs_component"] = err(dp[:, nprobe:], dp64[:, nprobe:])
            e["note"] = "characteristic-wise TENO5 (Roe-average eigenvectors per face) in the 2D three-pass form"
            res[name] = e
            continue
        if name != "fp64":
            e["speedup_vs_fp64"] = round(w64 / w, 3)
            e["acoustic_err_r50_vs_fp64"] = err(dp[:, :nprobe], dp64[:, :nprobe])
            e["acoustic_err_r10_vs_fp64"] = err(dp[:, nprobe:], dp64[:, nprobe:])
        if rec is not None:
            k50, k10 = min(rec["r50"].shape[0], dp.shape[0]), min(rec["r10"].shape[0], dp.shape[0])
            e["acoustic_err_r50_vs_oracle"] = err(dp[:k50, :nprobe], rec["r50"][:k50])
            e["acoustic_err_r10_vs_oracle"] = err(dp[:k10, nprobe:], rec["r10"][:k10])
        if name.startswith("learned32"):
            e["significant_side_frac"] = round(fr["significant"], 4)
            e["fallback_side_frac"] = round(fr["fallback"], 4)
            if name == "learned32":
                e["training"] = {"harvested_sides": int(F.shape[0]), "adam_steps": 4000,
                                 "final_loss": round(losses[-1], 4), "seconds": round(t_train, 1)}
            else:
                e["note"] = "keep patterns from each step's first stage, reused by its other two stages"
        res[name] = e
    res["c5_flapping_plate"] = flapping_plate(net, nsteps=plate_steps)
    progress("C5 rigid plate done")
    res["c5_flexible_plate_m1"] = flapping_plate(net, nsteps=plate_steps, flexible=True, mass_ratio=1.0)
    progress("C5 flexible plate, mass ratio 1, done")
    res["c5_flexible_plate"] = flapping_plate(net, nsteps=plate_steps, flexible=True)
    progress("C5 flexible plate, mass ratio 5, done")
    res["hovering_insect"] = hovering_insect(net, nsteps=plate_steps)
    progress("hovering insect done")
    res["run"] = {"steps": nsteps, "probes_per_ring": nprobe, "probe_every": every,
                  "max_probe_dp_r50": float(dp64[:, :nprobe].abs().max()),
                  "max_probe_dp_r10": float(dp64[:, nprobe:].abs().max()),
                  "oracle_record": rec is not None,
                  "note": "whole run from the uniform start (the configured 2000 steps and their continuation "
                          "until the start-up wave crosses the radius-50 ring), probe launches included in the "
                          "timing; errors are relative L2 over probes x samples, against the oracle's record "
                          "(radius 10: its first 2000 steps) and against the FP64 GPU run"}
    return res


def flapping_plate(net, nsteps=None, every=10, flexible=False, mass_ratio=5.0):
    """Config 5's plate at 1024^2 from the uniform stream over one flapping period
    (nsteps=None; 21,110 steps at CFL 0.5), rigid with the paper's prescribed heave and pitch
    or (flexible=True) following the flexible plate, which each step's marker forces load
    (explicit coupling: the force read-out synchronises every step); probes on a radius-3
    ring.  See moving_body_forms."""
    from paper_1905_00182_amd import workloads as W

    case = (W.config5_flexible(n=1024, mass_ratio=mass_ratio) if flexible else W.config5(n=1024)).with_(
        probes=W.ring_probes(64, 3.0))
    if nsteps is None:
        nsteps = int(round(1.0 / case.extra["plate"]["f"] / case.dt))
    return moving_body_forms(case, W.plate_kinematics, net, nsteps, every, flexible)


def hovering_insect(net, nsteps=None, every=10):
    """The hovering insect at 800^2 (50 cells per wing length) from rest over one flapping
    period (nsteps=None; 8000 steps); probes on a radius-5 ring.  See moving_body_forms."""
    from paper_1905_00182_amd import workloads as W

    case = W.insect()
    if nsteps is None:
        nsteps = int(round(1.0 / case.extra["insect"]["f"] / case.dt))
    return moving_body_forms(case, W.insect_kinematics, net, nsteps, every, False)


def moving_body_forms(case, kinematics, net, nsteps, every=10, flexible=False):
    """FP64 TENO5 against the FP32 precision form and the learned form with the selector once
    per step on a case whose markers move every step (positions and velocities set before
    each step by kinematics(case, t), or by the flexible plate; one step call per step
    continuing the previous one's state).  Delta p on the case's probes every `every` steps;
    errors are relative L2 over probes x samples against FP64."""
    import numpy as np
    import torch

    from paper_1905_00182_amd import fsa
    from paper_1905_00182_amd import workloads as W

    nsteps -= nsteps % every
    Q0 = torch.from_numpy(W.uniform_state(case)).cuda()
    runs = {}
    for name, prec, stride in (("fp64", "fp64", 1), ("mixed32", "mixed32", 1), ("learned32_stride3", "learned32", 3)):
        c = case.with_(precision=prec, extra={**case.extra, "selector_stride": stride})
        s = fsa.Solver(c, nan_check=flexible)      # (a coupled run reports a blow-up)
        if net is not None and prec == "learned32":
            s.mlp_set(net, 0.8)
        plate = fsa.Plate(c) if flexible else None
        Q = Q0.clone()
        nsamp = nsteps // every
        dps = torch.empty((nsamp, s.np), dtype=torch.float64, device=Q.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(nsamp):
            if flexible:     # the coupling loop inside the library
                try:
                    plate.coupled_steps(s, Q, c.dt, every, resume=k > 0)
                except fsa.FsaError as e:
                    s.close()
                    plate.close()
                    return {"grid": list(case.n[:2]), "form": name, "nonfinite_after_step": k * every,
                            "error": str(e), "mass_ratio": case.extra["flex"]["rho_s"]}
            else:
                for m in range(every):
                    s.set_marker_kinematics(*kinematics(c, (k * every + m) * c.dt))
                    if k == 0 and m == 0:
                        s.rk3_step(Q, c.dt)
                    else:
                        s.rk3_steps_resume(Q, c.dt)
            s.probe_dp(Q, out=dps[k])
        torch.cuda.synchronize()
        runs[name] = (time.perf_counter() - t0, dps)
        if flexible:
            X, _ = plate.markers()
            Xr, _ = kinematics(c, nsteps * c.dt)
            runs[name] += (float(np.abs(X - Xr).max()),)
            plate.close()
        s.close()
    w64, dp64 = runs["fp64"][:2]
    wm, dpm = runs["mixed32"][:2]
    wl, dpl = runs["learned32_stride3"][:2]
    cs = case.ncell * 3 * nsteps
    return {"grid": list(case.n[:2]), "steps": nsteps, "markers": int(case.markers["X"].shape[1]),
            **({"mass_ratio": case.extra["flex"]["rho_s"]} if flexible else {}),
            "probes": int(dp64.shape[1]), "probe_every": every,
            "fp64": {"value": round(cs / w64 / 1e6, 1), "unit": "Mcell-stage/s",
                     "ms_per_step": round(w64 / nsteps * 1e3, 4)},
            "mixed32": {"value": round(cs / wm / 1e6, 1), "unit": "Mcell-stage/s",
                        "ms_per_step": round(wm / nsteps * 1e3, 4), "speedup_vs_fp64": round(w64 / wm, 3),
                        "acoustic_err": float(torch.linalg.norm(dpm - dp64) / torch.linalg.norm(dp64))},
            "learned32_stride3": {"value": round(cs / wl / 1e6, 1), "unit": "Mcell-stage/s",
                                  "ms_per_step": round(wl / nsteps * 1e3, 4),
                                  "speedup_vs_fp64": round(w64 / wl, 3),
                                  "acoustic_err": float(torch.linalg.norm(dpl - dp64) / torch.linalg.norm(dp64))},
            "max_probe_dp": float(dp64.abs().max()),
            **({"plate_max_bend_fp64": runs["fp64"][2], "plate_max_bend_learned": runs["learned32_stride3"][2]}
               if flexible else {}),
            "acoustic_err_first_2000_steps": {
                k: float(torch.linalg.norm(d[:2000 // every] - dp64[:2000 // every]) / torch.linalg.norm(dp64[:2000 // every]))
                for k, d in (("mixed32", dpm), ("learned32_stride3", dpl))},
            "note": "markers moved before every step, one step call per step (continuing the "
                    "previous call's state)"}


def blocks(case, Q0, nsteps=200, nblocks=4):
    """The benchmark case in `nblocks` slabs on one GPU (fsa_mb_*, bit for bit the single
    context's result) against one context: ms per step of each, and whether the states
    agree bitwise after the run."""
    import torch

    from paper_1905_00182_amd import fsa

    import numpy as np

    s = fsa.Solver(case)
    Q = Q0.clone()
    s.rk3_steps(Q, case.dt, 2)
    s.set_state(np.zeros((case.dim, s.nm)), 0.0, 0)     # (as the blocks' scatter: a fresh start)
    Q = Q0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.rk3_steps(Q, case.dt, nsteps)
    torch.cuda.synchronize()
    w1 = time.perf_counter() - t0
    s.close()
    m = fsa.MultiBlock(case, nblocks)
    m.scatter(Q0)
    m.rk3_steps(case.dt, 2)
    m.scatter(Q0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.rk3_steps(case.dt, nsteps)
    torch.cuda.synchronize()
    wb = time.perf_counter() - t0
    same = bool(torch.equal(m.gather(), Q))
    m.close()
    return {"blocks": nblocks, "steps": nsteps, "ms_per_step_single": round(w1 / nsteps * 1e3, 4),
            "ms_per_step_blocks": round(wb / nsteps * 1e3, 4), "overhead": round(wb / w1 - 1.0, 4),
            "bitwise_equal": same,
            "note": "slabs along y, each with 4 halo rows per neighbour recomputed, halo copies and the "
                    "cross-block wave-speed maximum after every stage"}


# Algorithmic work and traffic of one 3D cell-stage (the 2D count carried to three directions
# and five components: 30 reconstructions, nine velocity derivatives, six stress components).
ALGO_FLOPS_3D = {"teno5": 2938, "weno5js": 2398}
ALGO_BYTES_3D = 106.7


def three_d(steps=3):
    """Rates of the 3D path on the sphere cases (256^3 FP64 in both schemes, 384^3 precision
    form): `steps` steps after one warm-up step, inputs resident on the device."""
    import torch

    from paper_1905_00182_amd import fsa
    from paper_1905_00182_amd import workloads as W

    out = {}
    for name, case in (("c3_256_teno5_fp64", W.config3(n=256, scheme="teno5")),
                       ("c3_256_weno5js_fp64", W.config3(n=256, scheme="weno5js")),
                       ("c3_256_teno5_fp64_characteristic", W.config3(n=256, scheme="teno5").with_(
                           variables="characteristic")),
                       ("c4_384_teno5_mixed32", W.config4(n=384))):
        Q = torch.from_numpy(W.config3_state(case)).cuda()
        s = fsa.Solver(case)
        s.rk3_steps(Q, case.dt, 1)
        s.timing(True)
        s.timing_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.rk3_steps(Q, case.dt, steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms, nl = s.timing_read()
        s.close()
        stage_ms = kms / max(nl, 1)
        out[name] = {"value": round(case.ncell * 3 * steps / wall / 1e6, 1), "unit": "Mcell-stage/s",
                     "ms_per_step": round(wall / steps * 1e3, 3),
                     "stage_kernels_ms_per_stage": round(stage_ms, 3)}
        if case.variables == "component" and stage_ms > 0:
            # the whole 3D stage (stress, face and stage passes) against the FP64 (C3) or FP32
            # (C4, its reconstruction's type) vector peak, at the method's algorithmic work
            flops = ALGO_FLOPS_3D[case.scheme]
            achieved = flops * case.ncell / (stage_ms * 1e-3) / 1e12
            peak = 78.6 if case.precision == "fp64" else 157.3
            out[name]["roofline"] = {
                "bound": "alu", "kernels": "the stage's passes", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "algo_flops_per_cell_stage": flops,
                "hbm_frac_algorithmic": round(ALGO_BYTES_3D * case.ncell / (stage_ms * 1e-3) / 8e12, 4)}
        del Q
        torch.cuda.empty_cache()
        progress(f"3D {name}: {out[name]['value']} Mcell-stage/s")
    return out


C3_RECORDS = {sch: os.path.join(ROOT, "tests", "golden", f"c3_oracle_run_{sch}.npz") for sch in ("teno5", "weno5js")}


def sphere_acoustics(nsteps=None):
    """The sphere cases' acoustic pressure at full size, at the 64 probes on the radius-4 sphere
    every 5 steps over the configured 500 steps: C4 (384^3) in the precision form against the
    same run in FP64, and C3 (256^3, TENO5 and WENO5-JS) in both forms against the CPU
    oracle's records of those runs (tests/golden/c3_oracle_run_<scheme>.npz, when present)."""
    import numpy as np
    import torch

    from paper_1905_00182_amd import fsa
    from paper_1905_00182_amd import workloads as W

    def run(case, steps):
        s = fsa.Solver(case)
        Q = torch.from_numpy(W.config3_state(case)).cuda()
        dp = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps // 5):
            s.rk3_steps(Q, case.dt, 5) if k == 0 else s.rk3_steps_resume(Q, case.dt, 5)
            dp.append(s.probe_dp(Q))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.close()
        del Q
        torch.cuda.empty_cache()
        return torch.stack(dp).cpu().numpy(), wall

    def err(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    out = {}
    c4 = W.config4(n=384)
    steps = nsteps or c4.steps
    dp64, w64 = run(c4.with_(precision="fp64"), steps)
    dp32, w32 = run(c4, steps)
    out["c4_384"] = {"steps": steps, "probes": int(dp64.shape[1]), "probe_every": 5,
                     "max_probe_dp_rel_p_inf": float(np.abs(dp64).max() / c4.prim_inf[4]),
                     "fp64_ms_per_step": round(w64 / steps * 1e3, 3),
                     "mixed32_ms_per_step": round(w32 / steps * 1e3, 3),
                     "acoustic_err_mixed32_vs_fp64": err(dp32, dp64)}
    progress(f"C4 384^3 acoustics: precision form vs FP64 {out['c4_384']['acoustic_err_mixed32_vs_fp64']:.2e}")
    for sch, path in C3_RECORDS.items():
        if not os.path.exists(path):
            continue
        rec = np.load(path)
        c3 = W.config3(n=256, scheme=sch)
        k = min(int(rec["steps"]), nsteps or c3.steps) // int(rec["every"])
        d64, _ = run(c3, k * 5)
        d32, _ = run(c3.with_(precision="mixed32"), k * 5)
        o = rec["dp"][:k]
        out[f"c3_256_{sch}"] = {"steps": k * 5, "max_probe_dp_rel_p_inf": float(np.abs(o).max() / c3.prim_inf[4]),
                                "acoustic_err_fp64_vs_oracle": err(d64, o),
                                "acoustic_err_mixed32_vs_oracle": err(d32, o),
                                "acoustic_err_mixed32_vs_fp64": err(d32, d64)}
        progress(f"C3 256^3 {sch} acoustics vs the oracle's record: FP64 "
                 f"{out[f'c3_256_{sch}']['acoustic_err_fp64_vs_oracle']:.2e}, precision form "
                 f"{out[f'c3_256_{sch}']['acoustic_err_mixed32_vs_oracle']:.2e}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the full-run comparison of the FP64, FP32 and FP32+learned forms")
    ap.add_argument("--variant-steps", type=int, default=4000,
                    help="steps of the full runs (default 4000: the configured 2000 and their continuation until "
                         "the start-up wave crosses the radius-50 ring)")
    ap.add_argument("--plate-steps", type=int, default=None,
                    help="steps of the flapping-plate and hovering-insect runs (default: one flapping period)")
    ap.add_argument("--scheme", default="teno5", choices=["teno5", "weno5js"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (counter calibration)")
    ap.add_argument("--only-3d", action="store_true",
                    help="only the 3D sphere-case rates, --steps steps each (for profiling the 3D kernels)")
    ap.add_argument("--only-sphere-acoustics", action="store_true",
                    help="only the sphere cases' full-size acoustic errors (C4 precision form vs FP64, C3 vs the "
                         "oracle's records)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the solver has no "
              "multi-GPU domain decomposition.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1905_00182_amd import fsa, workloads as W

    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 8, "copy_probe_bytes_written": b.numel() * 8,
                          "launches": 3}), flush=True)
        return
    if args.only_3d:
        print(json.dumps({"three_d": three_d(args.steps)}), flush=True)
        return
    if args.only_sphere_acoustics:
        print(json.dumps({"sphere_acoustics": sphere_acoustics()}), flush=True)
        return
    case = W.config2()
    if args.scheme != case.scheme:
        case = case.with_(scheme=args.scheme)
    Q0 = torch.from_numpy(W.config2_state(case)).cuda()

    def run(c):
        Q = Q0.clone()
        s = fsa.Solver(c)
        if args.warmup > 0:
            s.rk3_steps(Q, c.dt, args.warmup)
        s.sync()
        s.timing(True)
        s.timing_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.rk3_steps(Q, c.dt, args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms, launches = s.timing_read()
        s.timing(False)
        s.sync()
        return wall, kms, launches, Q, s

    wall, kms, launches, Q64, s = run(case)
    progress(f"headline: {args.steps} steps in {wall:.3f} s")
    cell_stages = case.ncell * 3 * args.steps
    value = cell_stages / wall / 1e6
    per_launch_ms = kms / max(launches, 1)
    flops_launch = ALGO_FLOPS_2D[case.scheme] * case.ncell
    achieved = flops_launch / (per_launch_ms * 1e-3) / 1e12
    traffic = traffic_from_profile(case.ncell)
    out = {
        "metric": "Mcell-stage updates/s (2D FP64 TENO5 + IB, SSP-RK3)",
        "value": round(value, 3),
        "unit": "Mcell-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"c2_rotating_cylinder_{case.n[0]}x{case.n[1]}_{case.scheme}_ib_fp64",
            "grid": [case.n[0], case.n[1]],
            "scheme": case.scheme,
            "markers": int(case.markers["X"].shape[1]),
            "re": 150,
            "mach": 0.2,
            "dt": case.dt,
        },
        "hbm_gbps_algorithmic": round(value * 1e6 * ALGO_BYTES_2D / 1e9, 1),
        "hbm_frac_algorithmic": round(value * 1e6 * ALGO_BYTES_2D / 1e9 / PEAK_HBM_GBPS, 4),
        "roofline": {
            "bound": "alu",
            "kernel": f"k_stage2d<{case.scheme.upper()}>",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
            "traffic": traffic,
            "kernel_ms_per_launch": round(per_launch_ms, 4),
            "launches": launches,
            "algo_flops_per_cell_stage": ALGO_FLOPS_2D[case.scheme],
        },
        "cpu_baseline": None,
    }
    if not args.no_variants:
        out["variants"] = variants(case, Q0, args.variant_steps, plate_steps=args.plate_steps)
        out["variants"]["three_d"] = three_d()
        out["variants"]["sphere_acoustics"] = sphere_acoustics()
        out["variants"]["c2_blocks"] = blocks(case, Q0)
        progress("blocks done")
    if not args.no_cpu and args.cpu_steps > 0:
        progress("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
