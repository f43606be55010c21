"""Plant plausible mistakes in a copy of the oracle and check that the pins fail.

Each mutant is the oracle source with one textual change (a dropped carry, a
missing correction step, a wrong index or bound), compiled on the CPU into a
temporary library.  The pin battery below must reject every one of them, which
shows the pins in test_oracle_pins.py are sharp enough to catch such slips.
"""
import ctypes
import os
import random
import subprocess
import sys

import numpy as np
import pytest

from conftest import ROOT, read_golden
from test_oracle_pins import ADD_BACK_CASES

SRC = os.path.join(ROOT, "oracle", "rsa_oracle.c")
U32P = ctypes.POINTER(ctypes.c_uint32)

MUTANTS = {
    "mul_drops_carry": ("k = t >> 32;", "k = 0;"),
    "no_add_back": ("if (t < 0) {", "if (0) {"),
    "no_qhat_correction": ("qhat -= 1;", "break;"),
    "skips_top_bit": ("for (int bit = top; bit >= 0; --bit)",
                      "for (int bit = top - 1; bit >= 0; --bit)"),
    "unnormalise_wrong_index": ("(uwork[i] >> s) | (uwork[i + 1] << (32 - s))",
                                "(uwork[i] >> s) | (uwork[i] << (32 - s))"),
    "no_normalisation": ("int s = __builtin_clz(v[n - 1]);", "int s = 0;"),
    "drops_squaring": ("modmul(c, a, a, a, n);", "(void)0;"),
    "one_mod_one": ("if (!(nl == 1 && n[0] == 1)) a[0] = 1;", "a[0] = 1;"),
    "borrow_sign": ("borrow = t >> 32;                 /* 0 or -1 */", "borrow = 0;"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    mutated = src.replace(old, new)
    c = tmp_path / (name + ".c")
    so = tmp_path / (name + ".so")
    c.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-pthread", "-w", str(c), "-o", str(so)],
                   check=True)
    L = ctypes.CDLL(str(so))
    L.oracle_modexp.argtypes = [U32P] * 4 + [ctypes.c_int]
    L.oracle_bn_mod.argtypes = [U32P, U32P, ctypes.c_int, U32P, ctypes.c_int]
    L.oracle_bn_mul.argtypes = [U32P, U32P, ctypes.c_int, U32P, ctypes.c_int]
    return L


def _span(x, k):
    return np.array([(x >> (32 * i)) & 0xFFFFFFFF for i in range(k)], dtype=np.uint32)


def _val(a):
    return sum(int(w) << (32 * i) for i, w in enumerate(a.tolist()))


def _p(a):
    return a.ctypes.data_as(U32P)


def _modexp(L, g, x, n):
    k = max(1, (max(g, x, n).bit_length() + 31) // 32)
    out = np.zeros(k, dtype=np.uint32)
    a, b, c = _span(g, k), _span(x, k), _span(n, k)
    L.oracle_modexp(_p(out), _p(a), _p(b), _p(c), k)
    return _val(out)


def _pins(L):
    """The pin battery: the paper's values, brute force and library checks."""
    g = read_golden("fig4_naive_trace.txt")
    assert _modexp(L, int(g["g"]), int(g["e"]), int(g["m"])) == 445
    for msg in range(0, 187, 5):                         # Section 3.4 key
        assert _modexp(L, _modexp(L, msg, 7, 187), 23, 187) == msg
    assert _modexp(L, 5, 0, 1) == 0
    rng = random.Random(11)
    for _ in range(60):
        n = rng.getrandbits(rng.randint(33, 400)) | 1
        m, e = rng.getrandbits(n.bit_length()), rng.getrandbits(rng.randint(1, 200))
        assert _modexp(L, m, e, n) == pow(m, e, n)
    for u, v in ADD_BACK_CASES:
        ku, kv = (u.bit_length() + 31) // 32, (v.bit_length() + 31) // 32
        r = np.zeros(kv, dtype=np.uint32)
        L.oracle_bn_mod(_p(r), _p(_span(u, ku)), ku, _p(_span(v, kv)), kv)
        assert _val(r) == u % v
    for _ in range(60):
        u, v = rng.getrandbits(rng.randint(64, 900)), rng.getrandbits(rng.randint(40, 300)) | 1
        ku, kv = (u.bit_length() + 31) // 32, (v.bit_length() + 31) // 32
        r = np.zeros(kv, dtype=np.uint32)
        L.oracle_bn_mod(_p(r), _p(_span(u, ku)), ku, _p(_span(v, kv)), kv)
        assert _val(r) == u % v
        w = np.zeros(ku + kv, dtype=np.uint32)
        L.oracle_bn_mul(_p(w), _p(_span(u, ku)), ku, _p(_span(v, kv)), kv)
        assert _val(w) == u * v


def test_unmutated_oracle_passes(tmp_path):
    L = _build(tmp_path, "clean", "/* D1:", "/* D1:")
    _pins(L)


def _run_battery(so_path):
    """Child-process entry: load a mutant library and run the pin battery."""
    L = ctypes.CDLL(so_path)
    L.oracle_modexp.argtypes = [U32P] * 4 + [ctypes.c_int]
    L.oracle_bn_mod.argtypes = [U32P, U32P, ctypes.c_int, U32P, ctypes.c_int]
    L.oracle_bn_mul.argtypes = [U32P, U32P, ctypes.c_int, U32P, ctypes.c_int]
    _pins(L)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    """The battery runs in a child process: a mutant may also loop for ever
    (a quotient estimate that is never corrected) or crash; a time-out or a
    crash counts as caught, a clean exit does not."""
    old, new = MUTANTS[name]
    _build(tmp_path, name, old, new)
    so = str(tmp_path / (name + ".so"))
    code = ("import sys; sys.path[:0] = [%r, %r]; import test_oracle_mutants as t; "
            "t._run_battery(%r)" % (os.path.join(ROOT, "tests"), ROOT, so))
    try:
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=20)
        caught = r.returncode != 0
    except subprocess.TimeoutExpired:
        caught = True
    assert caught, "mutant %s passed every pin" % name
