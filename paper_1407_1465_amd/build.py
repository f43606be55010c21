"""Build librsagpu.so for gfx950 with hipcc (in-tree, next to this file).

The kernel instances are spread over one translation unit per padded limb
width (csrc/kern_s<S>.hip) so they compile in parallel; rsagpu.hip holds the
host side.  Objects go to csrc/_build/ (not tracked)."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "librsagpu.so")
# the integer-multiply issue-rate probe the roofline is measured against
PEAK_SRC = os.path.join(HERE, "peak", "mulpeak.hip")
PEAK_LIB = os.path.join(HERE, "libmulpeak.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def deps():
    return sources() + glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(CSRC, "*.def")) + \
        [os.path.join(ROOT, "include", "rsagpu.h")]


def peak_deps():
    return [PEAK_SRC, os.path.join(ROOT, "include", "mulpeak.h")]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _compile(src: str, extra) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra) + ["-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on %s" % src)
    return obj


def _link(objs, out: str, verbose: bool) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-z,defs"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed (%d)" % r.returncode)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, out: str = LIB, extra=(), jobs: int = 0) -> str:
    """Compile every HIP source and link librsagpu.so, and the multiply
    probe libmulpeak.so beside it (always recompiles)."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources() + [PEAK_SRC]
    jobs = jobs or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), srcs))
    _link(objs[-1:], PEAK_LIB, verbose)
    return _link(objs[:-1], out, verbose)


def stale() -> bool:
    for lib, ds in ((LIB, deps()), (PEAK_LIB, peak_deps())):
        if not os.path.exists(lib):
            return True
        t = os.path.getmtime(lib)
        if any(os.path.getmtime(d) > t for d in ds if os.path.exists(d)):
            return True
    return False


if __name__ == "__main__":
    print(build(verbose=True))
