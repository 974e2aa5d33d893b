"""Build the HIP library libnyxhydro.so for gfx950 in-tree with hipcc.

Translation units:
  nyx_step.hip  twice: FP64 stages (no contraction) and FP32-mixed stages;
  nyx_util.hip  CFL reduction, dt finalisation, ghost fills (no contraction);
  nyx_fill.hip  ghost fill of an AMR level: planning, copies, coarse-fine
                interpolation (no contraction);
  nyx_sync.hip  two-level synchronisation: planning, reflux, average-down
                (no contraction);
  nyx_gravity.hip  gravity input: cloud-in-cell deposit, multigrid Poisson
                solve, centred gradient (no contraction);
  nyx_abi.cpp   the C ABI (validation, plans, dispatch).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnyxhydro.so")
ARCH = os.environ.get("NYX_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]

UNITS = [
    ("nyx_step.hip", "nyx_step_fp64.o", ["-DNYX_PREC_FP64", "-ffp-contract=off"]),
    # -amdgpu-mfma-vgpr-form: the network's MFMA accumulators live in VGPRs,
    # so reading them back costs no v_accvgpr_read per value
    ("nyx_step.hip", "nyx_step_mixed.o", ["-DNYX_PREC_MIXED", "-ffp-contract=on",
                                          "-fno-hip-fp32-correctly-rounded-divide-sqrt",
                                          "-mllvm", "-amdgpu-mfma-vgpr-form"]),
    ("nyx_mlp.hip", "nyx_mlp.o", ["-ffp-contract=on", "-mllvm", "-amdgpu-mfma-vgpr-form"]),
    ("nyx_util.hip", "nyx_util.o", ["-ffp-contract=off"]),
    ("nyx_fill.hip", "nyx_fill.o", ["-ffp-contract=off"]),
    ("nyx_sync.hip", "nyx_sync.o", ["-ffp-contract=off"]),
    ("nyx_gravity.hip", "nyx_gravity.o", ["-ffp-contract=off"]),
    ("nyx_abi.cpp", "nyx_abi.o", ["-ffp-contract=off", "-x", "hip"]),
]


def _compile(unit):
    src, obj, flags = unit
    cmd = ["hipcc"] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build() -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
        [os.path.join(BUILD, o) for o in objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
