"""CPU replay of the GPU sliding-window schedule.

The exponentiation kernels with 2 or 4 lanes per group run a left-to-right
sliding window per group: a two-word bit buffer refilled one word ahead, a
leading window that initialises A from the odd-power table, then one
Montgomery product per slot (squaring, or product with T[k] = x^(2k+1)).
This replays exactly those steps on the exponent alone (A's exponent doubles
on a squaring and grows by 2k+1 on a table product) and checks that the
schedule reaches e, stays within the table, and does the expected number of
products.  The GPU parity tests check the kernels' results themselves.
"""
import os
import random
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


class ExpBits:
    def __init__(self, words):
        self.words = words
        self.kw = 0
        self.bits = 0
        self.pre = 0

    def word(self, k):
        return self.words[k] if 0 <= k < len(self.words) else 0

    def start(self, top):
        self.kw = top >> 5
        self.bits = (self.word(self.kw) << 32) | self.word(self.kw - 1)
        self.pre = self.word(self.kw - 2)

    def seek(self, pos):
        if pos >= 0 and (pos >> 5) < self.kw:
            self.bits = ((self.bits << 32) | self.pre) & ((1 << 64) - 1)
            self.kw -= 1
            self.pre = self.word(self.kw - 2)

    def field(self, hi, lo):
        off = lo - 32 * (self.kw - 1)
        assert 0 <= off and hi - lo < 32 and hi - 32 * (self.kw - 1) < 64
        return (self.bits >> off) & ((1 << (hi - lo + 1)) - 1)


def schedule(e, w):
    """Returns (exponent reached, squarings, table products, table size used)."""
    words = [(e >> (32 * i)) & 0xFFFFFFFF for i in range((e.bit_length() + 31) // 32 + 1)]
    eb = ExpBits(words)
    ebits = e.bit_length()
    pos = ebits - 1
    st = {"sq": 0, "mi": -1, "pos": pos}

    def next_window():
        p = st["pos"]
        eb.seek(p)
        off = p - 32 * (eb.kw - 1)
        assert 32 <= off <= 63
        if ((eb.bits >> off) & 1) == 0:
            st.update(sq=1, mi=-1, pos=p - 1)
            return
        lo0 = max(p - w + 1, 0)
        v = eb.field(p, lo0)
        tz = (v & -v).bit_length() - 1
        v >>= tz
        st.update(sq=p - (lo0 + tz) + 1, mi=v >> 1, pos=lo0 + tz - 1)

    acc = 0                       # exponent of A (A = x^acc)
    nsq = nmul = 0
    top_mi = -1
    if st["pos"] >= 0:
        eb.start(st["pos"])
        next_window()
        acc = 2 * st["mi"] + 1
        top_mi = max(top_mi, st["mi"])
        st.update(sq=0, mi=-1)
        if st["pos"] >= 0:
            next_window()
    while st["sq"] > 0 or st["mi"] >= 0:
        if st["sq"] == 0 and st["mi"] >= 0:
            acc += 2 * st["mi"] + 1
            top_mi = max(top_mi, st["mi"])
            nmul += 1
            st["mi"] = -1
        else:
            acc *= 2
            nsq += 1
            st["sq"] -= 1
        if st["sq"] == 0 and st["mi"] < 0 and st["pos"] >= 0:
            next_window()
    return acc, nsq, nmul, top_mi


EDGE = [1, 2, 3, 5, 7, 65537, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, (1 << 64) - 1, 1 << 63,
        (1 << 1024) - 1, 1 << 1023, (1 << 1023) + 1, int("10" * 512, 2), int("1000" * 256, 2)]


@pytest.mark.parametrize("w", [2, 3, 4, 5, 6])
def test_schedule_reaches_exponent(w):
    rng = random.Random(w)
    cases = EDGE + [rng.getrandbits(rng.choice([17, 31, 32, 33, 63, 64, 65, 512, 1024, 2048])) | 1
                    for _ in range(200)]
    for e in cases:
        acc, nsq, nmul, top_mi = schedule(e, w)
        assert acc == e, (e, w)
        assert top_mi < (1 << (w - 1))               # within the odd-power table
        # every bit below the leading window costs exactly one squaring
        assert nsq <= e.bit_length() - 1


def table_size(e, w):
    """Odd powers the kernel builds: all 2^(w-1), or for exponents of at most
    64 bits the largest index the schedule uses plus one (its pre-scan)."""
    if e.bit_length() > 64:
        return 1 << (w - 1)
    return schedule(e, w)[3] + 1 if e else 0


@pytest.mark.parametrize("w", [2, 3, 4, 5])
def test_short_exponent_table_and_count(w):
    # 65537 = 2^16 + 1: x alone, 16 squarings and one product (binary method)
    acc, nsq, nmul, top = schedule(65537, w)
    assert (acc, nsq, nmul, top) == (65537, 16, 1, 0)
    assert table_size(65537, w) == 1
    import bench
    assert bench.sliding_window_montmuls(65537, w) == 17
    rng = random.Random(100 + w)
    for _ in range(200):
        e = rng.getrandbits(rng.choice([3, 17, 40, 64, 65, 200, 1024])) | 1
        acc, nsq, nmul, top = schedule(e, w)
        ts = table_size(e, w)
        assert top < ts <= (1 << (w - 1))
        assert bench.sliding_window_montmuls(e, w) == nsq + nmul + (ts if ts > 1 else 0)


def test_schedule_zero_exponent():
    assert schedule(0, 4)[:3] == (0, 0, 0)


def test_sliding_saves_products_on_1024_bit_exponents():
    """For random 1024-bit exponents the sliding window with w = 4 (8 odd
    powers, the LDS of a fixed 3-bit window) needs ~10% fewer products than
    the fixed 3-bit window (1023 squarings + 341 products)."""
    rng = random.Random(1)
    tot = 0
    for _ in range(50):
        e = rng.getrandbits(1024) | (1 << 1023)
        acc, nsq, nmul, _ = schedule(e, 4)
        assert acc == e
        tot += nsq + nmul + 8                         # + table (x^2 and 7 products)
    fixed = (1024 // 3) * 4 + 8                      # (ceil(1024/3) - 1) * (3 + 1) + 2^3 (approx.)
    assert tot / 50 < 0.93 * fixed
