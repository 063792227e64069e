"""Build the HIP library (gfx950) and its host emulator, in-tree.

  liblbfreeze.so       the C-ABI library (include/lbfreeze.h): kernels for
                       float32 and float64 plus the host API
  liblbfreeze_emu.so   host emulator of the step and reverse-step kernels
                       (CPU tests only)
  lbf_emu_sanitize     sanitizer driver of the emulator (CPU tests only)
  lbf_emu_adj_sanitize sanitizer driver of the emulated reverse step (CPU
                       tests only)

Usage: ``python -m paper_2603_22902_amd.build`` or ``build()``.  Every call
recompiles.  The kernels are compiled with packed-fp32 instructions
disabled; the float64 unit also without floating-point contraction.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "liblbfreeze.so")
EMU = os.path.join(HERE, "liblbfreeze_emu.so")
EMU_SAN = os.path.join(HERE, "lbf_emu_sanitize")
EMU_ADJ_SAN = os.path.join(HERE, "lbf_emu_adj_sanitize")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
DEV_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-I", INCLUDE,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
HOST_FLAGS = ["--offload-host-only", "-std=c++17", "-fPIC", "-I", INCLUDE,
              "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, emulator: bool = True) -> str:
    with tempfile.TemporaryDirectory(prefix="lbf_build_") as tmp:
        units = [("lbf_api.hip", []), ("lbf_kernels_f32.hip", []),
                 ("lbf_kernels_f32_ilp.hip", ["-mllvm", "--amdgpu-sched-strategy=max-ilp"]),
                 ("lbf_kernels_f64.hip", ["-ffp-contract=off"]), ("lbf_kernels_mix.hip", [])]
        objs = []
        jobs = []
        for src, extra in units:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            objs.append(obj)
            jobs.append([HIPCC, *DEV_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
        if emulator:
            jobs.append([HIPCC, *HOST_FLAGS, "-O2", "-shared", os.path.join(CSRC, "lbf_emu.hip"),
                         os.path.join(CSRC, "lbf_emu_adj.hip"), "-o", EMU + ".tmp"])
            jobs.append([HIPCC, *HOST_FLAGS, "-O1", "-g", "-DLBF_EMU_MAIN",
                         "-Xarch_host", "-fsanitize=address",
                         "-Xarch_host", "-fsanitize=undefined",
                         "-fno-omit-frame-pointer", os.path.join(CSRC, "lbf_emu.hip"),
                         "-o", EMU_SAN + ".tmp"])
            jobs.append([HIPCC, *HOST_FLAGS, "-O1", "-g", "-DLBF_EMU_ADJ_MAIN",
                         "-Xarch_host", "-fsanitize=address",
                         "-Xarch_host", "-fsanitize=undefined",
                         "-fno-omit-frame-pointer", os.path.join(CSRC, "lbf_emu_adj.hip"),
                         "-o", EMU_ADJ_SAN + ".tmp"])
        with ThreadPoolExecutor(max_workers=min(len(jobs), 6)) as ex:
            list(ex.map(lambda c: _run(c, verbose), jobs))
        _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"], verbose)
        os.replace(LIB + ".tmp", LIB)
        if emulator:
            os.replace(EMU + ".tmp", EMU)
            os.replace(EMU_SAN + ".tmp", EMU_SAN)
            os.replace(EMU_ADJ_SAN + ".tmp", EMU_ADJ_SAN)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, emulator="--no-emu" not in sys.argv)
    print(LIB)
