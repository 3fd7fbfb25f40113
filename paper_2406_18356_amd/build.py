"""Builds libmsr.so (HIP, gfx950) in-tree: one object per transform length,
the host API, one shared library next to this file.

    python -m paper_2406_18356_amd.build [--jobs J]

MSR_HIPCC_FLAGS (environment) adds hipcc flags, e.g. kernel switches such
as -DMSR_TW_PRELOAD_INV=1; MSR_OFFLOAD_ARCH overrides gfx950.
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmsr.so")
LENGTHS = [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]

ARCH = os.environ.get("MSR_OFFLOAD_ARCH", "gfx950")
CXXFLAGS = [
    "-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
# extra hipcc flags for experiments (e.g. -DMSR_ROW_PINGPONG=0), space separated
CXXFLAGS += os.environ.get("MSR_HIPCC_FLAGS", "").split()


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + out)
    return out


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = []
    for L in LENGTHS:
        obj = os.path.join(BUILD, f"ops_{L}.o")
        units.append([cc, *CXXFLAGS, f"-DMSR_L={L}", "-c", os.path.join(CSRC, "ops_inst.hip"), "-o", obj])
    for name in ("msr_api", "persist", "unet"):
        units.append([cc, *CXXFLAGS, "-c", os.path.join(CSRC, name + ".hip"), "-o", os.path.join(BUILD, name + ".o")])
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, units))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [u[-1] for u in units]
    tmp = LIB + ".tmp"
    _run([cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose))


if __name__ == "__main__":
    sys.exit(main())
