"""The host side of the library under AddressSanitizer.

The host code builds every table the kernels index: shell pairs, class
lists, groups, bra blocks, tiles, block tasks and their LDS row columns.  This
test builds fk_host.cpp with AddressSanitizer on the host side only (the GPU
code is not instrumented), links it with the library's kernel objects from
the last build, and in a separate process -- the sanitizer runtime preloaded,
PyTorch kept out -- builds the lists of C20H42, an s-f system, a batch of
three molecules and (H2O)32 (800 functions: large enough for the XCD-region
order of the work items) under four schedules (defaults, block tasks for every lane
class that can take them, the team alternatives of the lane classes, no
block tasks), checks every kernel address with fk_check_indices, and
requires the process to end cleanly.  Contexts without a device, so no GPU
is needed."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2407_21445_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DRIVER = r'''
import sys, time
sys.modules["torch"] = None
sys.path.insert(0, sys.argv[1])
sys.path.insert(1, sys.argv[2])
sys.path.insert(2, sys.argv[3])
import paper_2407_21445_amd as fk
from synth import workloads as wl
from synth import geometry as geom
from test_oracle import _rand_sys
wide = [(1, 0, 1, 0), (1, 1, 0, 0), (1, 1, 1, 0), (2, 0, 0, 0), (2, 0, 1, 0), (2, 1, 0, 0), (2, 1, 1, 0)]
alts = [((1, 1, 1, 0), 3), ((2, 0, 1, 0), 6), ((2, 1, 0, 0), 6), ((3, 0, 1, 0), 10), ((3, 1, 0, 0), 10)]
spdf = _rand_sys(41, lmax=3, natom=4, kmax=2)
systems = (("c20h42", wl.c20h42_631gs()), ("spdf", spdf),
           ("batch", wl.batch([wl.water4_sto3g(), wl.alkane_sys(2, "6-31gs-type"), spdf])),
           ("water32", wl.make_system(geom.water_sphere(32, wl.SEED + 3), "ccpvdz-type")))
for name, s in systems:
    for variant in ("default", "wide", "lanes", "off"):
        c = fk.FockJK(device=-1).set_system(s)
        if variant == "wide":
            for w in wide:
                c.set_class_block_tasks(*w, True)
        if variant == "lanes":
            for cls, n in alts:
                c.set_class_lanes(*cls, n)
        c.build_quartets(tau=1e-10, tau_prim=1e-12, block_tasks=(variant != "off"))
        c.check_indices()
        nt = sum(x["block_tasks"] > 0 for x in c.stats()["classes"])
        print(name, variant, nt, flush=True)
        c.close()
print("driver done")
'''


def _asan_runtime():
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return cands[-1] if cands else None


def test_host_tables_under_address_sanitizer(tmp_path):
    objs = sorted(glob.glob(os.path.join(PKG, "_build", "*.o")))
    objs = [o for o in objs if os.path.basename(o) != "fk_host.o"]
    rt = _asan_runtime()
    if not os.path.exists(HIPCC) or rt is None or len(objs) < 14:
        pytest.skip("needs hipcc, the sanitizer runtime and the kernel objects of a build")
    host_o = str(tmp_path / "fk_host_asan.o")
    # the sanitizer goes to the host compilation only (-Xarch_host before each option)
    cc = [HIPCC, "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
          "-DFK_BUILD_MAXL=3", "-I" + os.path.join(ROOT, "include"),
          "-c", os.path.join(PKG, "csrc", "fk_host.cpp"), "-o", host_o]
    r = subprocess.run(cc, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    pkg = tmp_path / "pkg" / "paper_2407_21445_amd"
    pkg.mkdir(parents=True)
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
            "-Xarch_host", "-shared-libasan", "-o", str(pkg / "libfockjk.so"), host_o] + objs + \
           ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocsolver", "-lrocblas"]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    shutil.copy(os.path.join(PKG, "__init__.py"), pkg / "__init__.py")
    drv = tmp_path / "drive.py"
    drv.write_text(DRIVER)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([sys.executable, str(drv), str(tmp_path / "pkg"), ROOT, os.path.join(ROOT, "tests")],
                       capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "driver done" in r.stdout and "AddressSanitizer" not in out, out[-6000:]
    lines = [l.split() for l in r.stdout.splitlines() if len(l.split()) == 3]
    got = {(a, b): int(n) for a, b, n in lines}
    assert got[("c20h42", "wide")] > got[("c20h42", "default")] > got[("c20h42", "off")] == 0
    assert got[("water32", "wide")] > got[("water32", "default")] > got[("water32", "off")] == 0
