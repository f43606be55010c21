"""The compiled headline kernel (k_crt<36,2,29>, 2048-bit CRT halves) keeps
its Montgomery products as one v_mad_u64_u32 per 32x29-bit limb product.

A change elsewhere in a kernel (the Montgomery set-up, for instance) can make
the compiler hold the modulus limbs as 64-bit values and lower every m*n[j]
as a 64x32-bit product (two multiply-adds and two moves), which doubles the
kernel's time without changing any result.  This test compiles the
translation unit for gfx950 (hipcc cross-compiles without a GPU) and checks
the counts in the kernel's assembly."""
import os
import re
import shutil
import subprocess
from collections import Counter

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1407_1465_amd", "csrc")


@pytest.mark.slow
def test_headline_kernel_products_are_single_multiply_adds(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = os.path.join(CSRC, "kern_b29_s36.hip")
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "--cuda-device-only", "-S", src, "-o",
           str(tmp_path / "k.s")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    text = (tmp_path / "k.s").read_text()
    start = re.search(r"^_ZN6rsagpu5k_crtILi36ELi2ELi29E\w*:", text, re.M)
    assert start, "k_crt<36,2,29> not found"
    body = text[start.end():text.index(".Lfunc_end", start.end())]
    ops = Counter(m.group(1) for m in re.finditer(r"^\s+([a-z_0-9]+)", body, re.M))
    mads, movs = ops["v_mad_u64_u32"], ops["v_mov_b32_e32"]
    # one multiply-add per limb product: 36 x 18 for m*n and the squaring's
    # share per product, in the hot loop and its copies; moves stay a small
    # fraction of them
    assert mads > 5000
    assert movs < 0.2 * mads, "v_mov_b32: %d for %d v_mad_u64_u32" % (movs, mads)
