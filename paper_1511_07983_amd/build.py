"""Build libko.so in-tree with hipcc for gfx950.

    python paper_1511_07983_amd/build.py

compiles csrc/ko_host.cpp, ko_sim.hip, ko_lanes.hip, ko_rounds.hip, ko_select.hip and
ko_hw.hip into
paper_1511_07983_amd/libko.so,
and csrc/ko_nn.hip (the learned surrogate) into paper_1511_07983_amd/libko_nn.so.
Host code is built with -ffp-contract=off so the binary64 scores of the
launch-order heuristic are evaluated exactly as written.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libko.so")
LIB_NN = os.path.join(HERE, "libko_nn.so")
ARCH = os.environ.get("KO_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
    "-ffp-contract=off",
]
DEVICE = [
    f"--offload-arch={ARCH}",
    # never emit packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# Per-source device flags (none at present).
EXTRA = {}


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    host_o = os.path.join(objdir, "ko_host.o")
    sim_o = os.path.join(objdir, "ko_sim.o")
    _run([HIPCC, *COMMON, "-x", "hip", *DEVICE, "-c", os.path.join(CSRC, "ko_host.cpp"), "-o", host_o])
    _run([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, "ko_sim.hip"), "-o", sim_o])
    sel_o = os.path.join(objdir, "ko_select.o")
    _run([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, "ko_select.hip"), "-o", sel_o])
    hw_o = os.path.join(objdir, "ko_hw.o")
    _run([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, "ko_hw.hip"), "-o", hw_o])
    lanes_o = os.path.join(objdir, "ko_lanes.o")
    _run([HIPCC, *COMMON, *DEVICE, *EXTRA.get("ko_lanes.hip", []), "-c", os.path.join(CSRC, "ko_lanes.hip"),
          "-o", lanes_o])
    rounds_o = os.path.join(objdir, "ko_rounds.o")
    _run([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, "ko_rounds.hip"), "-o", rounds_o])
    tmp = LIB + ".tmp"
    _run([HIPCC, *DEVICE, "-shared", "-fPIC", host_o, sim_o, sel_o, hw_o, lanes_o, rounds_o, "-o", tmp])
    os.replace(tmp, LIB)
    nn_o = os.path.join(objdir, "ko_nn.o")
    _run([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, "ko_nn.hip"), "-o", nn_o])
    tmp = LIB_NN + ".tmp"
    _run([HIPCC, *DEVICE, "-shared", "-fPIC", nn_o, "-o", tmp])
    os.replace(tmp, LIB_NN)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
