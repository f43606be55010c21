"""Seeded input generators: determinism, key consistency and message ranges."""
import math

import numpy as np
import pytest

from paper_1407_1465_amd import workloads as W


def test_splitmix64_reference_values():
    # SplitMix64 with seed 0: the published first outputs of the generator.
    r = W.SplitMix64(0)
    assert [r.next64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                              0x06C45D188009454F]
    blk = W.splitmix64_block(0, 0, 3)
    assert blk.tolist() == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert W.splitmix64_block(1234, 5, 4).tolist() == \
        [W._mix64((1234 + i * W._GAMMA) & W.MASK64) for i in range(6, 10)]


@pytest.mark.parametrize("bits", [64, 128, 512, 1024])
def test_key_consistency(bits):
    k = W.make_key(bits, 99 + bits)
    k.check()
    assert k.n.bit_length() == bits and k.p.bit_length() == k.q.bit_length() == bits // 2
    assert k.p > k.q and math.gcd(k.e, (k.p - 1) * (k.q - 1)) == 1
    # deterministic for a seed
    assert W.make_key(bits, 99 + bits) == k


def test_key_cache_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setenv("RSAGPU_KEY_CACHE", str(tmp_path))
    a = W.make_keys(256, 5, 3, processes=1)
    b = W.make_keys(256, 5, 3, processes=1)
    assert a == b and len(list(tmp_path.iterdir())) == 1
    assert len({k.n for k in a}) == 3


def test_small_primes_and_mr():
    rng = W.SplitMix64(3)
    primes = set(W._small_primes(5000))
    for c in range(2, 5000):
        assert W.is_probable_prime(c, rng, 8) == (c in primes)
    # Carmichael numbers and a strong pseudoprime to base 2
    for c in (561, 41041, 825265, 321197185, 2047, 3215031751):
        assert not W.is_probable_prime(c, rng, 8)
    assert W.is_probable_prime((1 << 127) - 1, rng, 16)
    assert not W.is_probable_prime((1 << 128) + 1, rng, 16)


def test_uniform_below_range_and_determinism():
    n = W.make_key(512, 17).n
    a = W.uniform_below(n, 2000, 42)
    b = W.uniform_below(n, 2000, 42)
    assert np.array_equal(a, b) and a.shape == (2000, 16)
    vals = W.limbs_to_ints(a)
    assert all(0 <= v < n for v in vals)
    # the top bits are spread over [0, n): chi-square on 8 equal bins
    bins = np.bincount([v * 8 // n for v in vals], minlength=8)
    chi2 = ((bins - 250.0) ** 2 / 250.0).sum()
    assert chi2 < 24.3            # 7 dof, p = 0.001
    # a small modulus in a wider limb field
    small = W.uniform_below(1000, 500, 1, limbs=2)
    assert small.shape == (500, 2) and max(W.limbs_to_ints(small)) < 1000


def test_limb_conversion():
    vals = [0, 1, (1 << 64) - 1, 12345678901234567890123]
    arr = W.ints_to_limbs(vals, 3)
    assert arr.dtype == np.uint32 and arr.shape == (4, 3)
    assert W.limbs_to_ints(arr) == vals


def test_workload_shapes_small():
    w = W.workload_c1(count=64)
    assert w.msgs.shape == (64, 2) and w.limbs == 2 and len(w.keys) == 1
    assert all(m < w.keys[0].n for m in W.limbs_to_ints(w.msgs))
    w3 = W.single_size_workload("t", 256, 4, 40, 7)
    assert w3.key_of.tolist() == [i % 4 for i in range(40)]
    for i, m in enumerate(W.limbs_to_ints(w3.ctxt)):
        assert m < w3.keys[i % 4].n


def test_paper_table_keys():
    """The keys of the paper's Section 10 experiment: Table 1's n = 131 * 137
    with the Section 2 example exponent 131 (whose printed partner 137 is not
    its inverse: 131 * 137 mod phi(n) = 267), Table 2's n = 1009 * 509 (the
    caption's 1005 is composite); d inverts e modulo phi(n) and messages
    stay in 0..800."""
    k1, k2 = W.PAPER_TABLE_KEYS[1], W.PAPER_TABLE_KEYS[2]
    assert (k1.n, k2.n) == (17947, 513581)
    assert (131 * 137) % ((k1.p - 1) * (k1.q - 1)) == 267
    assert k1.d == 14171
    for k in (k1, k2):
        assert (k.e * k.d) % ((k.p - 1) * (k.q - 1)) == 1
        assert all(pow(pow(m, k.e, k.n), k.d, k.n) == m for m in range(801))
    m = W.paper_table_messages(32768)
    assert m.shape == (32768, 1) and int(m.min()) == 0 and int(m.max()) == 800
    assert np.array_equal(m, W.paper_table_messages(32768))
    assert len(W.PAPER_TABLE_SIZES) == len(W.PAPER_TABLE_GPU_TIME[1]) == len(W.PAPER_TABLE_GPU_TIME[2])


def test_text_packets_match_section2_golden():
    """The packet codec against the packets printed for the Section 2
    example (tests/golden/packets_sec2.txt)."""
    import os
    golden = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "packets_sec2.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.rstrip("\n").split(" ", 1)
                golden[k] = v
    packets = [int(p) for p in golden["packets"].split()]
    assert W.text_to_packets(golden["text"]) == packets
    assert W.packets_to_text(packets) == golden["text"].replace(" ", "")
