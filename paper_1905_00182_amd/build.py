"""Build the gfx950 solver library paper_1905_00182_amd/libfsa.so from csrc/ with hipcc.

All device code is compiled with packed-FP32 instructions disabled (they are never emitted)
and with contraction of a multiply and an add into an FMA only within one source expression
(-ffp-contract=on): the rounding of a formula is then fixed by its source text, so kernels
that evaluate the same formula (the precision form's TENO5 and the learned form's fallback)
agree bit for bit whatever the surrounding code.  The C ABI is declared in include/fsa.h
(the solver) and include/fsa_plate.h (the flexible plate, host code) at the repository root.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfsa.so")
SOURCES = ["fsa_api.hip", "k_stage2d.hip", "k_stage3d.hip", "k_pass2d.hip", "k_ib.hip", "k_mlp.hip", "k_faces2d.hip",
           "k_nrbc.hip", "k_halo.hip", "plate.cpp"]
ARCH = os.environ.get("FSA_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [
        hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        "-o", LIB + ".tmp",
    ] + [os.path.join(CSRC, s) for s in SOURCES] + list(extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
