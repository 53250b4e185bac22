"""Build liblbm.so (HIP, gfx950) in-tree.

The step kernels are compiled once per population storage type (four
translation units) in parallel with the auxiliary kernels and the host
runtime, then linked into one shared library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbm.so")

ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse a*b+c only inside one expression: every inlined copy of the site
    # arithmetic (halo pass, main loop) then rounds identically
    "-ffp-contract=on",
    "-I", INCLUDE, "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-fvisibility=hidden",
]


def _units():
    units = [(os.path.join(CSRC, "step.hip"), f"step_st{k}.o", [f"-DLBM_ST={k}"]) for k in range(4)]
    units.append((os.path.join(CSRC, "aux.hip"), "aux.o", []))
    units.append((os.path.join(CSRC, "static_step.hip"), "static_step.o", []))
    units.append((os.path.join(CSRC, "lbm.cpp"), "lbm.o", ["-x", "hip"]))
    return units


def _compile(src, obj, extra):
    out = os.path.join(BUILD, obj)
    cmd = [HIPCC, *COMMON, *extra, "-c", src, "-o", out]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 target feature: harmless
    noise = [ln for ln in proc.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if proc.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n" + "\n".join(noise))
    return out, "\n".join(noise)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(_units()), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _compile(*u), _units()))
    objs = [r[0] for r in results]
    if verbose:
        for _, warn in results:
            if warn:
                print(warn, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{proc.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
