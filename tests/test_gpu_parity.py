"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Every result is compared element by element with the oracle on the same
seeded inputs, at sizes that span several waves and a ragged tail; at the
full workload sizes a seeded sample of outputs is checked against the oracle
and the whole batch against the round-trip property (M^e)^d mod n = M.
"""
import random

import numpy as np
import pytest

from paper_1407_1465_amd import workloads as W
from gpu_util import dev, host, oracle_modexp, crt_operands, full_operands

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_1465_amd import rsagpu  # noqa: E402  (fails loudly if the library is missing)

WIDTHS = [1, 2, 3, 4, 5, 8, 12, 16, 24, 31, 32, 48, 64, 96, 128]


def _random_case(rng, limbs, count):
    bits = 32 * limbs
    mods, bases, exps = [], [], []
    for i in range(count):
        nb = bits if i % 3 else rng.randint(2, bits)
        n = (rng.getrandbits(nb) | (1 << (nb - 1)) | 1)
        if i % 7 == 3:
            n = (1 << bits) - 1                     # top limb all ones
        mods.append(n)
        bases.append(rng.getrandbits(bits))         # may exceed n
        kind = i % 5
        if kind == 0:
            e = rng.getrandbits(bits)
        elif kind == 1:
            e = rng.getrandbits(rng.randint(1, 24))
        elif kind == 2:
            e = 65537
        elif kind == 3:
            e = rng.getrandbits(max(1, bits // 2))
        else:
            e = rng.getrandbits(bits) | (1 << (bits - 1))
        exps.append(e)
    return [W.ints_to_limbs(v, limbs) for v in (bases, exps, mods)]


@pytest.mark.parametrize("limbs", WIDTHS)
def test_modexp_random_vs_oracle(limbs):
    plan = rsagpu.get_plan(limbs, 0)
    ng = 64 // plan.lanes_per_op
    count = 2 * ng + 5 if limbs >= 64 else 3 * ng + 5        # several waves + a ragged tail
    rng = random.Random(1000 + limbs)
    B, E, M = _random_case(rng, limbs, count)
    out = host(rsagpu.modexp(dev(B), dev(E), dev(M)))
    want = oracle_modexp(B, E, M)
    bad = np.nonzero((out != want).any(axis=1))[0]
    assert bad.size == 0, "limbs=%d: %d mismatches, first at %d" % (limbs, bad.size, bad[0])
    assert rsagpu.device_errors() == 0


@pytest.mark.parametrize("limbs", [2, 32, 64])
def test_modexp_special_cases(limbs):
    rng = random.Random(7 + limbs)
    bits = 32 * limbs
    n = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    e = rng.getrandbits(bits) | 1
    cases = [
        (5, 0, n), (0, 0, n), (12345, 1, n), (n + 5, 1, n), (0, e, n), (1, e, n),
        (n - 1, e, n), (n - 1, e - 1, n), (n - 1, 2, n), (2, e, 3), (5, 3, 3),
        ((1 << bits) - 1, e, n), ((1 << bits) - 1, (1 << bits) - 1, (1 << bits) - 1),
        (7, 5, 1),                                      # n = 1: result 0, not an error
    ]
    B, E, M = (W.ints_to_limbs([c[i] for c in cases], limbs) for i in range(3))
    out = host(rsagpu.modexp(dev(B), dev(E), dev(M)))
    got = W.limbs_to_ints(out)
    assert got == [pow(b, x, m) for b, x, m in cases]
    assert got == W.limbs_to_ints(oracle_modexp(B, E, M))
    assert rsagpu.device_errors() == 0


def test_modexp_data_errors():
    limbs = 4
    cases = [(3, 5, 10), (3, 5, 0), (3, 5, 97), (2, 2, 1 << 64)]
    B, E, M = (W.ints_to_limbs([c[i] for c in cases], limbs) for i in range(3))
    out = W.limbs_to_ints(host(rsagpu.modexp(dev(B), dev(E), dev(M))))
    assert out == [0, 0, pow(3, 5, 97), 0]
    assert rsagpu.device_errors() == 3
    assert rsagpu.device_errors() == 0


def test_modexp_in_place_and_empty():
    limbs = 8
    rng = random.Random(3)
    B, E, M = _random_case(rng, limbs, 70)
    want = oracle_modexp(B, E, M)
    b = dev(B)
    rsagpu.modexp(b, dev(E), dev(M), out=b)
    assert np.array_equal(host(b), want)
    empty = dev(np.zeros((0, limbs), dtype=np.uint32))
    rsagpu.modexp(empty, empty, empty)


def test_workload_rsa64_full_size():
    """64-bit key, 4096 messages: encrypt and full-d decrypt, all checked."""
    w = W.workload_c1()
    k = w.keys[0]
    L = w.limbs
    n = full_operands(w.keys, w.key_of, L, "n")
    e = full_operands(w.keys, w.key_of, L, "e")
    d = full_operands(w.keys, w.key_of, L, "d")
    c = host(rsagpu.modexp(dev(w.msgs), dev(e), dev(n)))
    assert np.array_equal(c, oracle_modexp(w.msgs, e, n))
    m = host(rsagpu.modexp(dev(c), dev(d), dev(n)))
    assert np.array_equal(m, w.msgs)                       # round trip
    dec = host(rsagpu.modexp(dev(w.ctxt), dev(d), dev(n)))
    assert np.array_equal(dec, oracle_modexp(w.ctxt, d, n))
    assert W.limbs_to_ints(c[:4]) == [pow(x, k.e, k.n) for x in W.limbs_to_ints(w.msgs[:4])]


def test_workload_rsa1024_full_size():
    """1024-bit key, 65536 messages: every full-d decryption and every
    encryption against the oracle; the whole batch round-trips."""
    w = W.workload_c2()
    L = w.limbs
    n = full_operands(w.keys, w.key_of, L, "n")
    e = full_operands(w.keys, w.key_of, L, "e")
    d = full_operands(w.keys, w.key_of, L, "d")
    dec = host(rsagpu.modexp(dev(w.ctxt), dev(d), dev(n)))
    bad = np.nonzero((dec != oracle_modexp(w.ctxt, d, n)).any(axis=1))[0]
    assert bad.size == 0, "%d of %d decryptions differ, first %d" % (bad.size, len(dec), bad[0])
    c = rsagpu.modexp(dev(w.msgs), dev(e), dev(n))
    assert np.array_equal(host(c), oracle_modexp(w.msgs, e, n))
    m = host(rsagpu.modexp(c, dev(d), dev(n)))
    assert np.array_equal(m, w.msgs)


@pytest.mark.parametrize("bits,count", [(64, 300), (256, 130), (1024, 90), (2048, 70), (3072, 45), (4096, 45)])
def test_crt_vs_oracle_plain_decrypt(bits, count):
    """CRT decryption equals the oracle's plain C^d mod n on every element
    (3072- and 4096-bit halves run two wave pairs per workgroup: 45 messages
    are several workgroups and a ragged last one)."""
    keys = W.make_keys(bits, 77 + bits, 4) if bits < 3072 else W.make_keys(bits, W.SEED_BASE + 4, 16)[:4]
    L = keys[0].limbs
    key_of = np.arange(count) % 4
    rng = random.Random(bits)
    cs = [rng.randrange(keys[i % 4].n) for i in range(count)]
    cs[0], cs[1], cs[2] = 0, 1, keys[2].n - 1
    cs[3] = keys[3].p                                       # gcd(c, n) > 1
    cs[4] = keys[0].q * 5 % keys[0].n
    C = W.ints_to_limbs(cs, L)
    p, q, dp, dq, qi = crt_operands(keys, key_of, L)
    out = host(rsagpu.decrypt_crt(dev(C), dev(p), dev(q), dev(dp), dev(dq), dev(qi)))
    n = full_operands(keys, key_of, L, "n")
    d = full_operands(keys, key_of, L, "d")
    want = oracle_modexp(C, d, n)
    bad = np.nonzero((out != want).any(axis=1))[0]
    assert bad.size == 0, "%d mismatches, first at %d" % (bad.size, bad[0] if bad.size else -1)
    assert rsagpu.device_errors() == 0


def test_crt_rejects_p_not_greater_than_q():
    keys = W.make_keys(128, 5, 1)
    k = keys[0]
    L = k.limbs
    h = L // 2
    C = W.ints_to_limbs([5, 7], L)
    # element 0 swapped (p < q), element 1 correct
    p = W.ints_to_limbs([k.q, k.p], h)
    q = W.ints_to_limbs([k.p, k.q], h)
    dp = W.ints_to_limbs([k.dq, k.dp], h)
    dq = W.ints_to_limbs([k.dp, k.dq], h)
    qi = W.ints_to_limbs([pow(k.p, -1, k.q), k.qinv], h)
    out = W.limbs_to_ints(host(rsagpu.decrypt_crt(dev(C), dev(p), dev(q), dev(dp), dev(dq), dev(qi))))
    assert out == [0, pow(7, k.d, k.n)]
    assert rsagpu.device_errors() == 1


@pytest.mark.parametrize("bits", [256, 2048])
def test_crt_grouped_by_key_with_data_errors(bits):
    """Several workgroups of messages under a few keys in random order (the
    launch regroups them by key, so waves hold one key's halves, or several
    keys' where groups meet) with invalid elements scattered through them:
    every valid element equals the oracle, every invalid one is 0 and
    counted once."""
    keys = W.make_keys(bits, 91 + bits, 3)
    L = keys[0].limbs
    h = L // 2
    count = 197
    rng = np.random.default_rng(bits)
    key_of = rng.integers(0, 3, count)
    r = random.Random(bits + 1)
    C = W.ints_to_limbs([r.randrange(keys[k].n) for k in key_of], L)
    p, q, dp, dq, qi = crt_operands(keys, key_of, L)
    bad_swap, bad_even = 7, 140
    k = keys[key_of[bad_swap]]
    p[bad_swap], q[bad_swap] = W.ints_to_limbs([k.q], h)[0], W.ints_to_limbs([k.p], h)[0]
    k = keys[key_of[bad_even]]
    q[bad_even] = W.ints_to_limbs([k.q + 1], h)[0]
    out = host(rsagpu.decrypt_crt(dev(C), dev(p), dev(q), dev(dp), dev(dq), dev(qi)))
    want = oracle_modexp(C, full_operands(keys, key_of, L, "d"), full_operands(keys, key_of, L, "n"))
    want[bad_swap] = 0
    want[bad_even] = 0
    wrong = np.nonzero((out != want).any(axis=1))[0]
    assert wrong.size == 0, "%d mismatches, first at %d" % (wrong.size, wrong[0])
    assert rsagpu.device_errors() == 2


@pytest.mark.parametrize("bits,runs", [
    (256, [37, 64, 100, 1, 70, 129]),        # runs that are not whole waves: each starts a wave of its own
    (2048, [33, 31, 64, 5, 96]),
    (128, [1] * 600),                        # 600 keys: padded runs would not fit, the order stays dense
])
def test_crt_key_runs_of_any_length(bits, runs):
    """Messages under several keys, shuffled, with per-key counts that are
    not multiples of a wave's messages (the key-grouped order pads each
    key's run to whole waves where the padding fits the launch, and packs
    the runs back to back where it does not): every element equals the
    oracle, and the static-scratch call returns the same."""
    keys = W.make_keys(bits, 13 + bits + len(runs), len(runs))
    L = keys[0].limbs
    key_of = np.repeat(np.arange(len(runs)), runs)
    np.random.default_rng(bits).shuffle(key_of)
    r = random.Random(bits + 3)
    C = W.ints_to_limbs([r.randrange(keys[k].n) for k in key_of], L)
    ops = [dev(a) for a in crt_operands(keys, key_of, L)]
    out = host(rsagpu.decrypt_crt(dev(C), *ops))
    want = oracle_modexp(C, full_operands(keys, key_of, L, "d"), full_operands(keys, key_of, L, "n"))
    wrong = np.nonzero((out != want).any(axis=1))[0]
    assert wrong.size == 0, "%d mismatches, first at %d" % (wrong.size, wrong[0])
    static = host(rsagpu.decrypt_crt_static(dev(C), *ops, out=torch.empty_like(dev(C))))
    assert np.array_equal(static, out)
    assert rsagpu.device_errors() == 0


def _order_bucket(key, hl):
    """The plain CRT call's 16-bit grouping hash of a key (its words p[0],
    p[1], dp[0], dq[0]), restated here only to pick keys whose buckets meet."""
    m = 0xFFFFFFFF
    rotl = lambda x, r: ((x << r) | (x >> (32 - r))) & m
    p, dp, dq = (W.int_to_limbs(v, hl) for v in (key.p, key.dp, key.dq))
    h = (int(p[0]) * 0x9E3779B1) & m
    h ^= (((int(p[1]) if hl > 1 else 0) + 0x7F4A7C15) & m) * 0x85EBCA77 & m
    h = rotl(h, 13) ^ ((int(dp[0]) * 0xC2B2AE3D) & m)
    h = rotl(h, 11) ^ ((int(dq[0]) * 0x27D4EB2F) & m)
    h ^= h >> 15
    h = (h * 0x2C1B3C6D) & m
    h ^= h >> 12
    return h >> 16


def test_crt_keys_whose_buckets_meet():
    """Two keys whose grouping hashes meet (found among 400 seeded 256-bit
    keys), with 37 and 50 messages (not whole waves), shuffled with three
    other keys: the two share one run, so its waves hold both keys' halves
    and take the per-group schedule, and every element still equals the
    oracle's plain C^d mod n, through both CRT entry points."""
    pool = W.make_keys(256, 7777, 400)
    hl = pool[0].limbs // 2
    seen, pair = {}, None
    for i, k in enumerate(pool):
        b = _order_bucket(k, hl)
        if b in seen:
            pair = (seen[b], i)
            break
        seen[b] = i
    assert pair is not None, "no two seeded keys share a bucket"
    keys = [pool[pair[0]], pool[pair[1]], pool[0], pool[1], pool[2]]
    runs = [37, 50, 5, 64, 70]
    L = keys[0].limbs
    key_of = np.repeat(np.arange(len(keys)), runs)
    np.random.default_rng(7).shuffle(key_of)
    r = random.Random(8)
    C = W.ints_to_limbs([r.randrange(keys[k].n) for k in key_of], L)
    ops = [dev(a) for a in crt_operands(keys, key_of, L)]
    out = host(rsagpu.decrypt_crt(dev(C), *ops))
    want = oracle_modexp(C, full_operands(keys, key_of, L, "d"), full_operands(keys, key_of, L, "n"))
    wrong = np.nonzero((out != want).any(axis=1))[0]
    assert wrong.size == 0, "%d mismatches, first at %d" % (wrong.size, wrong[0])
    static = host(rsagpu.decrypt_crt_static(dev(C), *ops, out=torch.empty_like(dev(C))))
    assert np.array_equal(static, out)
    assert rsagpu.device_errors() == 0


def test_crt_two_pair_workgroups_for_two_lane_halves():
    """8736 1024-bit messages under 16 keys (546 per key, not whole waves):
    273 wave pairs of 2-lane halves, between one and two one-pair workgroups
    per CU, so the call runs two pairs per workgroup where the kernel's
    occupancy allows it, over a key order padded to whole waves.  Every
    element equals the oracle's plain C^d mod n."""
    count, nk = 8736, 16
    keys = W.make_keys(1024, W.SEED_BASE + 4, nk)
    L = keys[0].limbs
    key_of = np.arange(count) % nk
    C = np.zeros((count, L), dtype=np.uint32)
    for j, k in enumerate(keys):
        idx = np.nonzero(key_of == j)[0]
        C[idx] = W.uniform_below(k.n, idx.size, W.derive_seed(8736, j, 1), L)
    out = host(rsagpu.decrypt_crt(dev(C), *[dev(a) for a in crt_operands(keys, key_of, L)]))
    want = oracle_modexp(C, full_operands(keys, key_of, L, "d"), full_operands(keys, key_of, L, "n"))
    bad = np.nonzero((out != want).any(axis=1))[0]
    assert bad.size == 0, "%d mismatches, first at %d" % (bad.size, bad[0] if bad.size else -1)
    assert rsagpu.device_errors() == 0


@pytest.mark.parametrize("table", [1, 2])
def test_paper_table_keys_round_trip(table):
    """The paper's Section 10 experiment on one-word keys: every encryption
    of 32768 messages in 0..800 (and a ragged 300) equals Python's pow and
    the oracle, and decryption returns every message."""
    key = W.PAPER_TABLE_KEYS[table]
    for N in (300, 32768):
        msgs = W.paper_table_messages(N)
        e = np.full((N, 1), key.e, dtype=np.uint32)
        d = np.full((N, 1), key.d, dtype=np.uint32)
        n = np.full((N, 1), key.n, dtype=np.uint32)
        c = host(rsagpu.modexp(dev(msgs), dev(e), dev(n)))
        assert [int(v) for v in c[:, 0]] == [pow(int(m), key.e, key.n) for m in msgs[:, 0]]
        if N == 300:
            assert np.array_equal(c, oracle_modexp(msgs, e, n))
        back = host(rsagpu.modexp(dev(c), dev(d), dev(n)))
        assert np.array_equal(back, msgs)
    assert rsagpu.device_errors() == 0


def test_section2_text_example_end_to_end():
    """Section 2's example flow on the GPU: "parallel encryption" as
    two-letter packets, encrypted with (e, n) = (131, 17947), decrypted with
    d = 14171 (the inverse of 131 mod phi(n); the printed 137 is not), back
    to the text."""
    key = W.PAPER_TABLE_KEYS[1]
    packets = W.text_to_packets("parallel encryption")
    N = len(packets)
    m = np.array(packets, dtype=np.uint32).reshape(N, 1)
    col = lambda v: np.full((N, 1), v, dtype=np.uint32)
    c = host(rsagpu.modexp(dev(m), dev(col(key.e)), dev(col(key.n))))
    assert [int(v) for v in c[:, 0]] == [pow(p, key.e, key.n) for p in packets]
    back = host(rsagpu.modexp(dev(c), dev(col(key.d)), dev(col(key.n))))
    assert W.packets_to_text([int(v) for v in back[:, 0]]) == "parallelencryption"


def test_workload_rsa2048_crt_full_size():
    """64 keys of 2048 bits, 16384 messages round-robin: every CRT decryption
    of the batch (one call, as the benchmark times it) and every e = 65537
    encryption against the oracle, plus the encrypt/decrypt round trip."""
    w = W.workload_c3()
    L = w.limbs
    p, q, dp, dq, qi = (dev(a) for a in crt_operands(w.keys, w.key_of, L))
    n = full_operands(w.keys, w.key_of, L, "n")
    d = full_operands(w.keys, w.key_of, L, "d")
    e = full_operands(w.keys, w.key_of, L, "e")
    dec = host(rsagpu.decrypt_crt(dev(w.ctxt), p, q, dp, dq, qi))
    bad = np.nonzero((dec != oracle_modexp(w.ctxt, d, n)).any(axis=1))[0]
    assert bad.size == 0, "%d of %d decryptions differ, first %d" % (bad.size, len(dec), bad[0])
    c = rsagpu.modexp(dev(w.msgs), dev(e), dev(n))
    assert np.array_equal(host(c), oracle_modexp(w.msgs, e, n))
    m = host(rsagpu.decrypt_crt(c, p, q, dp, dq, qi))
    assert np.array_equal(m, w.msgs)
    assert rsagpu.device_errors() == 0
