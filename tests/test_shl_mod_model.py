"""Host model of the kernels' rgrp_shl_mod (x * 2^c mod n in radix 2^29 over
a lane group, the step that moves R mod n and the R^2 ladder up by up to 28
bits at a time): the double-precision estimate of q = floor(y / n), summed
per lane from the top limb down and across the group's lanes in the kernel's
butterfly order, must never exceed floor(y / n) and must leave y - q n below
3n, so that the S-limb difference is exact and two subtractions of n make it
canonical.  Checked on random and edge-case moduli of every radix-2^29
width class, including moduli far shorter than the class."""
import math
import random

import pytest

B = 29
M = (1 << B) - 1
CLASSES = [(18, 2), (28, 4), (36, 2), (36, 4), (56, 8), (64, 16), (72, 4), (72, 8), (80, 16), (112, 8),
           (144, 16)]


def limbs(v, S):
    return [(v >> (B * i)) & M for i in range(S)]


def group_scaled(x, top, e, S, G):
    """Lane 0's value of rgrp_scaled: per-lane partial sums, then the xor
    butterfly (lane 0 adds lane o's running value for o = 1, 2, 4, ...)."""
    L = S // G
    parts = []
    for r in range(G):
        part = math.ldexp(float(top), B * S - e) if r == G - 1 else 0.0
        for j in range(L - 1, -1, -1):
            part += math.ldexp(float(x[r * L + j]), B * (r * L + j) - e)
        parts.append(part)
    o = 1
    while o < G:
        parts = [parts[r] + parts[r ^ o] for r in range(G)]
        o <<= 1
    return parts[0]


def shl_mod(xv, c, nv, S, G):
    bl = nv.bit_length()
    rn = 1.0 / group_scaled(limbs(nv, S), 0, bl, S, G)
    y = xv << c
    ylimbs = limbs(y & ((1 << (B * S)) - 1), S)
    top = y >> (B * S)
    qd = math.floor(group_scaled(ylimbs, top, bl, S, G) * rn) - 1.0
    q = int(qd) if qd > 0 else 0
    assert 0 <= q < (1 << 32)
    return y, q


@pytest.mark.parametrize("S,G", CLASSES)
def test_quotient_estimate_bounds(S, G):
    rng = random.Random(S * 100 + G)
    width = B * S - 10                         # n < 2^(B*S - 10), as every class guarantees
    cases = 0
    for _ in range(300):
        bits = rng.choice([width, width - 1, rng.randint(2, width), rng.randint(width - 64, width)])
        n = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
        for x in (rng.randrange(n), n - 1, 1, (1 << (n.bit_length() - 1)) % n):
            for c in (1, 13, 27, 28, rng.randint(1, 28)):
                y, q = shl_mod(x, c, n, S, G)
                assert q <= y // n, (S, G, n, x, c)
                r = y - q * n
                assert 0 <= r < 3 * n and r < (1 << (B * S))
                cases += 1
    assert cases > 1000


def test_quotient_near_integer_boundaries():
    """y / n just below and just above an integer (the cases where the
    estimate's rounding matters)."""
    S, G = 72, 4
    rng = random.Random(7)
    for _ in range(2000):
        n = rng.getrandbits(2048) | (1 << 2047) | 1
        k = rng.randrange(1, 1 << 28)
        for y in (k * n - 1, k * n, k * n + 1):
            c = 28
            x = y >> c
            if x >= n:
                continue
            yy, q = shl_mod(x, c, n, S, G)
            assert q <= yy // n and yy - q * n < 3 * n
