"""Builds libfockjk.so in-tree with hipcc for gfx950.

The class kernels are split over several translation units (one per bra pair
class) so that they compile in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfockjk.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          # packed FP32 instructions stay off (they are not needed by FP64 code)
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-variable", "-Wno-unused-function", "-Wno-unknown-warning-option"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout[-20000:])
    return r.stdout


def build(maxl: int = 3, jobs: int | None = None, verbose: bool = False, extra=()) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    defs = [f"-DFK_BUILD_MAXL={maxl}", f"-I{INCLUDE}"] + list(extra)
    units = []
    # the kernel file is compiled once per bra pair class (FK_ONLY_P selects it)
    for P in range(10):
        units.append((os.path.join(CSRC, "fk_kernels.hip"), os.path.join(BUILD, f"fk_kernels_p{P}.o"),
                      [f"-DFK_ONLY_P={P}"]))
    units.append((os.path.join(CSRC, "fk_kernels.hip"), os.path.join(BUILD, "fk_kernels_common.o"),
                  ["-DFK_ONLY_P=-1"]))
    # the McMurchie-Davidson J engine
    units.append((os.path.join(CSRC, "fk_kernels.hip"), os.path.join(BUILD, "fk_kernels_jeng.o"),
                  ["-DFK_ONLY_P=-2"]))
    units.append((os.path.join(CSRC, "fk_scf.hip"), os.path.join(BUILD, "fk_scf.o"), []))
    units.append((os.path.join(CSRC, "fk_guess.hip"), os.path.join(BUILD, "fk_guess.o"), []))
    units.append((os.path.join(CSRC, "fk_scf_batch.hip"), os.path.join(BUILD, "fk_scf_batch.o"), []))
    units.append((os.path.join(CSRC, "fk_host.cpp"), os.path.join(BUILD, "fk_host.o"), ["-x", "hip"]))
    cmds = [[HIPCC] + COMMON + defs + u[2] + ["-c", u[0], "-o", u[1]] for u in units]
    with cf.ThreadPoolExecutor(jobs) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for o in outs:
            if o.strip():
                print(o[-4000:])
    tmp = LIB + f".tmp{os.getpid()}"
    # rocSOLVER: the overlap eigen-decomposition of the canonical orthogonaliser
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + [u[1] for u in units] +
         ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocsolver", "-lrocblas"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    maxl = int(sys.argv[1]) if len(sys.argv) > 1 else 3
    print(build(maxl=maxl, verbose=True))
