"""Pins for the CPU oracle: each checks it against something other than itself.

* values the paper prints (Fig. 4 trace, the Section 3.4 key, the Section 2
  example key and packets), stored under tests/golden/ with citations;
* brute force: the naive repeated multiplication of Section 3.6.2 on tiny
  moduli, and exhaustive round trips for the toy key;
* Python's built-in integers (``*``, ``%``, three-argument ``pow``), an
  independent library implementation, on seeded random sizes and edge shapes;
* invariants: Fermat, Euler, the exponent-split identity of Section 6, and
  the special cases e = 0, e = 1, M = 0, M = 1, M = n - 1.
"""
import math
import random

import numpy as np
import pytest

import oracle
from conftest import read_golden
from paper_1407_1465_amd import workloads as W


# ---- paper values -----------------------------------------------------------

def test_fig4_naive_trace():
    g = read_golden("fig4_naive_trace.txt")
    base, e, m = int(g["g"]), int(g["e"]), int(g["m"])
    want = [int(v) for v in g["trace"].split()]
    got, trace = oracle.modexp_naive(base, e, m, trace=True)
    assert trace == want
    assert got == want[-1] == 445
    # the binary methods reach the same value
    assert oracle.modexp(base, e, m) == 445
    assert oracle.modexp(base, e, m, method="rtl") == 445


def test_toy_key_round_trip_exhaustive():
    k = {a: int(b) for a, b in read_golden("toy_key_sec3_4.txt").items()}
    assert k["p"] * k["q"] == k["n"]
    assert (k["p"] - 1) * (k["q"] - 1) == k["phi"]
    assert (k["e"] * k["d"]) % k["phi"] == 1
    for msg in range(k["n"]):
        c = oracle.modexp(msg, k["e"], k["n"])
        assert c == oracle.modexp_naive(msg, k["e"], k["n"])
        assert oracle.modexp(c, k["d"], k["n"]) == msg


def test_section2_example_key():
    g = read_golden("packets_sec2.txt")
    e, n, d_printed = int(g["e"]), int(g["n"]), int(g["d_printed"])
    packets = [int(p) for p in g["packets"].split()]
    # the packets are the a=00 .. z=25 code of the text, two letters each
    letters = g["text"].replace(" ", "")
    assert packets == [int("%02d%02d" % (ord(letters[2 * i]) - 97, ord(letters[2 * i + 1]) - 97))
                       for i in range(len(letters) // 2)]
    p, q = 131, 137
    assert p * q == n
    phi = (p - 1) * (q - 1)
    # The printed private exponent does not invert e (reading: encrypt-only
    # vector); the consistent one is e^-1 mod phi.
    assert (e * d_printed) % phi != 1
    d = pow(e, -1, phi)
    assert d == 14171
    for m in packets:
        c = oracle.modexp(m, e, n)
        assert c == pow(m, e, n)
        assert oracle.modexp(c, d, n) == m


# ---- brute force ------------------------------------------------------------

def test_naive_vs_binary_tiny_moduli():
    rng = random.Random(1)
    for _ in range(300):
        n = rng.randrange(1, 1 << 16)
        e = rng.randrange(0, 1 << 12)
        g = rng.randrange(0, 1 << 20)
        want = oracle.modexp_naive(g, e, n)
        assert oracle.modexp(g, e, n) == want, (g, e, n)
        assert oracle.modexp(g, e, n, method="rtl") == want, (g, e, n)


def test_naive_exhaustive_small_grid():
    n = 497
    for g in range(0, n, 7):
        for e in range(0, 40):
            assert oracle.modexp(g, e, n) == oracle.modexp_naive(g, e, n)


# ---- Python integers (independent library) ----------------------------------

def _edge_values(rng, limbs):
    bits = 32 * limbs
    return [
        (1 << bits) - 1,                        # all ones
        1 << (bits - 1),                        # top bit only
        ((1 << bits) - 1) ^ ((1 << 32) - 1),    # zero low limb
        (1 << (bits - 1)) | 1,
        rng.getrandbits(bits) | (1 << (bits - 1)),
        rng.getrandbits(bits - 1) + 1,
    ]


# Inputs for which the two-limb quotient estimate survives its correction
# test and the multiply-subtract goes negative, so the add-back step runs
# (found by searching 32-bit-limb shapes with a model of the estimate).
ADD_BACK_CASES = [
    (0x1000000000000000000000000, 0x10000000000000001),
    (0x7fffffff000000000000000000000000, 0x10000000000000001),
    (0xffffffff000000000000000000000000, 0x10000000000000001),
    (0x1000000010000000000000000, 0x10000000100000001),
    (0x2000000010000000000000000, 0x30000000000000001),
]


def test_bn_mul_and_mod_vs_python():
    rng = random.Random(2)
    for _ in range(400):
        a = rng.getrandbits(rng.randint(1, 2200))
        b = rng.getrandbits(rng.randint(1, 1100)) or 1
        assert oracle.bn_mul(a, b) == a * b
        assert oracle.bn_mod(a, b) == a % b


def test_knuth_d_edge_divisors():
    """Divisors and dividends that exercise the qhat estimate, its correction
    and the add-back step, against Python and the bit-serial remainder."""
    rng = random.Random(3)
    cases = []
    for limbs in (2, 3, 5, 8, 33):
        for v in filter(None, _edge_values(rng, limbs)):
            for qv in (1, (1 << 32) - 1, (1 << 64) - 1, rng.getrandbits(100)):
                for r in (0, v - 1, rng.randrange(v)):
                    cases.append((v * qv + r, v))
    cases += ADD_BACK_CASES
    for u, v in cases:
        assert oracle.bn_mod(u, v) == u % v
    for u, v in cases[:60]:
        assert oracle.bn_mod(u, v, slow=True) == u % v


def test_modexp_vs_pow_random_and_edges():
    rng = random.Random(4)
    for _ in range(150):
        limbs = rng.randint(1, 20)
        n = rng.getrandbits(32 * limbs) or 1
        g = rng.getrandbits(rng.randint(1, 32 * limbs))
        x = rng.getrandbits(rng.randint(0, 32 * limbs))
        assert oracle.modexp(g, x, n) == pow(g, x, n)
    for limbs in (1, 2, 4, 32):
        for n in filter(None, _edge_values(rng, limbs)):
            g, x = rng.getrandbits(32 * limbs), rng.getrandbits(32 * limbs)
            assert oracle.modexp(g, x, n) == pow(g, x, n)


# ---- invariants -------------------------------------------------------------

@pytest.mark.parametrize("bits", [64, 256, 512])
def test_fermat_euler_roundtrip(bits):
    key = W.make_key(bits, 1000 + bits)
    rng = random.Random(bits)
    phi = (key.p - 1) * (key.q - 1)
    for _ in range(6):
        a = rng.randrange(2, key.p - 1)
        assert oracle.modexp(a, key.p - 1, key.p) == 1            # Fermat
        assert oracle.modexp(a, key.p, key.p) == a
        b = rng.randrange(2, key.n - 1)
        if math.gcd(b, key.n) == 1:
            assert oracle.modexp(b, phi, key.n) == 1              # Euler
        m = rng.randrange(key.n)
        c = oracle.modexp(m, key.e, key.n)
        assert oracle.modexp(c, key.d, key.n) == m                 # round trip


def test_exponent_split_identity():
    """Section 6: M^e mod n = (M^(e-x) mod n * M^x mod n) mod n."""
    rng = random.Random(6)
    for _ in range(40):
        n = rng.getrandbits(200) | 1
        m = rng.randrange(n)
        e = rng.getrandbits(150)
        x = rng.randrange(e + 1)
        lhs = oracle.modexp(m, e, n)
        rhs = oracle.bn_mod(oracle.bn_mul(oracle.modexp(m, e - x, n), oracle.modexp(m, x, n)), n)
        assert lhs == rhs


def test_special_cases():
    rng = random.Random(7)
    for _ in range(30):
        n = rng.getrandbits(rng.randint(2, 300)) | 3
        m = rng.randrange(n)
        e = rng.getrandbits(100) | 2
        assert oracle.modexp(m, 0, n) == 1
        assert oracle.modexp(m, 1, n) == m
        assert oracle.modexp(m + n, 1, n) == m                     # base >= n is reduced
        assert oracle.modexp(0, e, n) == 0
        assert oracle.modexp(1, e, n) == 1
        assert oracle.modexp(n - 1, e, n) == (1 if e % 2 == 0 else n - 1)
        assert oracle.modexp(n - 1, e | 1, n) == n - 1
    assert oracle.modexp(5, 0, 1) == 0                             # n = 1
    assert oracle.modexp(0, 0, 7) == 1
    with pytest.raises(ZeroDivisionError):
        oracle.modexp(3, 3, 0)


# ---- batch driver -----------------------------------------------------------

def test_batch_driver_matches_pow():
    rng = random.Random(8)
    k = 5
    count = 37
    base = [rng.getrandbits(160) for _ in range(count)]
    exps = [rng.getrandbits(rng.randint(0, 160)) for _ in range(count)]
    mods = [rng.getrandbits(160) | 1 for _ in range(count)]
    B, E, M = (W.ints_to_limbs(v, k) for v in (base, exps, mods))
    out1, _, _ = oracle.modexp_batch(B, E, M, nthreads=1)
    out4, wall, used = oracle.modexp_batch(B, E, M, nthreads=4)
    assert used == 4 and wall >= 0
    assert np.array_equal(out1, out4)
    assert W.limbs_to_ints(out1) == [pow(b, e, m) for b, e, m in zip(base, exps, mods)]
    # shared exponent and modulus (stride 0)
    outs, _, _ = oracle.modexp_batch(B, E[3], M[5], nthreads=3)
    assert W.limbs_to_ints(outs) == [pow(b, exps[3], mods[5]) for b in base]
