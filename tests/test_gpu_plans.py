"""Every compiled kernel instance (limb radix, width, lanes per exponentiation)
against the CPU oracle, bit-exact, for both plain exponentiation and CRT
decryption.  Each instance is selected with rsa_set_plan and restored after."""
import os
import random
import re

import numpy as np
import pytest

from conftest import ROOT
from paper_1407_1465_amd import workloads as W
from gpu_util import dev, host, oracle_modexp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_1465_amd import rsagpu  # noqa: E402

DEF = os.path.join(ROOT, "paper_1407_1465_amd", "csrc", "instances.def")
INSTANCES = [tuple(map(int, m)) for m in re.findall(r"X\((\d+), (\d+), (\d+)\)", open(DEF).read())]
# radix-2^29 limb count -> the 32-bit width class it serves
CLASS_OF_S29 = {18: 16, 28: 24, 36: 32, 56: 48, 64: 48, 72: 64, 80: 64, 112: 96, 144: 128}


def width_class(B, S):
    return S if B == 32 else CLASS_OF_S29[S]


def window_for(B, S, G):
    for w in (3, 2):
        if (1 << w) * S * (64 // G) * 4 <= 64 * 1024:
            return w
    raise AssertionError("no window fits")


@pytest.fixture
def plan_guard():
    touched = []
    yield touched
    for limbs, kind in touched:
        rsagpu.set_plan(limbs, kind, 0, 0, 0)


@pytest.mark.parametrize("B,S,G", INSTANCES)
def test_instance_modexp(B, S, G, plan_guard):
    cls = width_class(B, S)
    rsagpu.set_plan(cls, 0, B, G, window_for(B, S, G))
    plan_guard.append((cls, 0))
    p = rsagpu.get_plan(cls, 0)
    assert (p.radix_bits, p.padded_limbs, p.lanes_per_op) == (B, S, G)
    rng = random.Random(B * 1000 + S * 10 + G)
    for limbs in sorted({cls, max(1, cls - 1)}):
        ng = 64 // G
        count = ng + 3 if cls >= 64 else 2 * ng + 3
        bits = 32 * limbs
        mods = [rng.getrandbits(bits) | (1 << (bits - 1)) | 1 for _ in range(count)]
        mods[1] = (1 << bits) - 1
        mods[2] = rng.getrandbits(bits // 2) | 1 | (1 << (bits // 2 - 1))   # short modulus
        bases = [rng.getrandbits(bits) for _ in range(count)]
        exps = [rng.getrandbits(rng.choice([bits, 17, bits // 3 + 1])) for _ in range(count)]
        exps[0] = 0
        exps[3] = 1
        Bv, Ev, Mv = (W.ints_to_limbs(v, limbs) for v in (bases, exps, mods))
        out = host(rsagpu.modexp(dev(Bv), dev(Ev), dev(Mv)))
        want = oracle_modexp(Bv, Ev, Mv)
        bad = np.nonzero((out != want).any(axis=1))[0]
        assert bad.size == 0, "B=%d S=%d G=%d limbs=%d: %d bad, first %d" % (B, S, G, limbs, bad.size, bad[0])
    assert rsagpu.device_errors() == 0


@pytest.mark.parametrize("B,S,G", INSTANCES)
def test_instance_modexp_shared_exponent(B, S, G, plan_guard):
    """Waves whose groups all carry the same exponent words (one key's
    exponent, a public exponent) run one schedule for the whole wave with
    symmetric squarings; a wave with one differing exponent, and the ragged
    last wave, must give the same results as the per-group schedule.  An
    exponent whose last window is its lowest bit alone (65537, 17) ends with
    one product by the base itself in place of the conversion out of the
    Montgomery domain: bases of any size below 2^(32 limbs), also far above a
    short modulus, must come out reduced."""
    cls = width_class(B, S)
    rsagpu.set_plan(cls, 0, B, G, window_for(B, S, G))
    plan_guard.append((cls, 0))
    rng = random.Random(B * 7 + S * 3 + G)
    limbs, bits, ng = cls, 32 * cls, 64 // G
    count = 2 * ng + 3
    mods = [rng.getrandbits(bits) | (1 << (bits - 1)) | 1 for _ in range(count)]
    mods[4] = (1 << bits) - 1
    bases = [rng.getrandbits(bits) for _ in range(count)]
    e1 = rng.getrandbits(bits) | (1 << (bits - 1))
    exps = [e1] * ng + [e1] * ng + [65537] * 3
    exps[ng + 5] = rng.getrandbits(bits)           # breaks the second wave's sharing
    cases = [(bases, exps, mods)]
    for e in (0, 1, 2, 3, 1 << (bits - 1), (1 << bits) - 1, 65537):
        cases.append((bases[:ng + 1], [e] * (ng + 1), mods[:ng + 1]))
    short = [rng.getrandbits(bits // 2) | 1 | (1 << (bits // 2 - 1)) for _ in range(ng + 1)]
    big = [(1 << bits) - 1 - rng.getrandbits(bits // 4) for _ in range(ng + 1)]
    for e in (65537, 17):
        cases.append((big, [e] * (ng + 1), short))
    for bs, es, ms in cases:
        Bv, Ev, Mv = (W.ints_to_limbs(v, limbs) for v in (bs, es, ms))
        out = host(rsagpu.modexp(dev(Bv), dev(Ev), dev(Mv)))
        want = oracle_modexp(Bv, Ev, Mv)
        bad = np.nonzero((out != want).any(axis=1))[0]
        assert bad.size == 0, "B=%d S=%d G=%d e[0]=%#x: %d bad, first %d" % (B, S, G, es[0], bad.size, bad[0])
    assert rsagpu.device_errors() == 0


# instances that serve CRT halves: up to the half of a 128-word modulus
CRT_INSTANCES = [i for i in INSTANCES if 64 // i[2] >= 2 and i[1] <= (64 if i[0] == 32 else 80)]


def test_wide_instances_have_no_crt_plan():
    for B, S, G in INSTANCES:
        if (B, S, G) not in CRT_INSTANCES and 64 // G >= 2:
            with pytest.raises(Exception):
                rsagpu.set_plan(width_class(B, S), 1, B, G, 2)


@pytest.mark.parametrize("B,S,G", CRT_INSTANCES)
def test_instance_crt(B, S, G, plan_guard):
    cls = width_class(B, S)
    rsagpu.set_plan(cls, 1, B, G, window_for(B, S, G))
    plan_guard.append((cls, 1))
    bits = 64 * cls
    keys = W.make_keys(bits, 4242 + bits, 2)
    L = keys[0].limbs
    h = L // 2
    ng = 64 // G                          # messages per workgroup
    count = 2 * ng + 3                    # key-ordered: at least one workgroup of one key
    rng = random.Random(S * G + B)
    key_of = np.arange(count) % 2
    cs = [rng.randrange(keys[k].n) for k in key_of]
    cs[0], cs[1] = 0, keys[1].n - 1
    C = W.ints_to_limbs(cs, L)

    def col(attr, width):
        return np.ascontiguousarray(W.ints_to_limbs([getattr(k, attr) for k in keys], width)[key_of])

    out = host(rsagpu.decrypt_crt(dev(C), dev(col("p", h)), dev(col("q", h)), dev(col("dp", h)),
                                  dev(col("dq", h)), dev(col("qinv", h))))
    want = oracle_modexp(C, col("d", L), col("n", L))
    bad = np.nonzero((out != want).any(axis=1))[0]
    assert bad.size == 0, "B=%d S=%d G=%d: %d bad" % (B, S, G, bad.size)
    assert rsagpu.device_errors() == 0


def test_autotune_installs_a_working_plan(plan_guard):
    plan_guard.append((32, 1))
    plan_guard.append((16, 0))
    best = rsagpu.autotune(64, 1, 0, 1024)
    assert rsagpu.get_plan(32, 1) == best
    best0 = rsagpu.autotune(16, 0, 17, 2048)
    assert rsagpu.get_plan(16, 0) == best0
    keys = W.make_keys(2048, 4242 + 2048, 2)
    L, h = keys[0].limbs, keys[0].limbs // 2
    key_of = np.arange(10) % 2
    rng = random.Random(5)
    C = W.ints_to_limbs([rng.randrange(keys[k].n) for k in key_of], L)

    def col(attr, width):
        return np.ascontiguousarray(W.ints_to_limbs([getattr(k, attr) for k in keys], width)[key_of])

    out = host(rsagpu.decrypt_crt(dev(C), dev(col("p", h)), dev(col("q", h)), dev(col("dp", h)),
                                  dev(col("dq", h)), dev(col("qinv", h))))
    assert np.array_equal(out, oracle_modexp(C, col("d", L), col("n", L)))
    assert rsagpu.device_errors() == 0


def ops_batch_vs_oracle(keys, kinds, count, seed):
    """count operations round-robin over `keys` (kind per op), through one
    rsa_ops_batch call, compared element by element with the oracle."""
    L = keys[0].limbs
    ks = rsagpu.KeySet(len(keys))
    for k in keys:
        ks.add(k.limbs, k.n, k.e, k.p, k.q, k.dp, k.dq, k.qinv)
    kid = np.arange(count) % len(keys)
    X = np.concatenate([W.uniform_below(keys[j].n, 1, W.derive_seed(seed, i), L) for i, j in enumerate(kid)])
    offs = np.arange(count, dtype=np.int64) * L
    ops = rsagpu.pack_ops(kinds, kid, offs, offs).cuda()
    out = torch.zeros(count * L, dtype=torch.int32, device="cuda")
    ws = torch.empty(rsagpu.ops_workspace_size(count), dtype=torch.uint8, device="cuda")
    rsagpu.ops_batch(ks, ops, dev(X.reshape(-1)), out, ws)
    got = host(out).reshape(count, L)
    exps = W.ints_to_limbs([keys[j].d if kd else keys[j].e for j, kd in zip(kid, kinds)], L)
    want = oracle_modexp(X, exps, W.ints_to_limbs([keys[j].n for j in kid], L))
    ks.close()
    return np.nonzero((got != want).any(axis=1))[0]


@pytest.mark.parametrize("bits,kind,count", [(2048, 2, 512), (4096, 3, 256), (512, 4, 16384)])
def test_autotune_ops_plans_install_working_plans(bits, kind, count, plan_guard):
    """rsa_autotune for the ops-batch kinds (2: encryption, 3: CRT half, 4:
    the CRT half of the widest class of a bulk batch of >= 16384 operations)
    installs a plan; a batch of real keys that takes that plan matches the
    oracle bit for bit."""
    L = bits // 32
    width = L if kind == 2 else L // 2
    plan_guard.append((width, kind))
    best = rsagpu.autotune(L, kind, 0, count)
    assert rsagpu.get_plan(width, kind) == best
    if bits == 512:
        keys = W.make_keys(512, 6161, 3)
    else:
        keys = W.make_keys(bits, W.SEED_BASE + 5, 256 if bits == 2048 else 64)[:3]
    kinds = np.full(count, 0 if kind == 2 else 1, dtype=np.int64)
    bad = ops_batch_vs_oracle(keys, kinds, count, 7000 + bits)
    assert bad.size == 0, "%d-bit kind %d plan %s: %d bad" % (bits, kind, best, bad.size)
    assert rsagpu.device_errors() == 0


def test_bulk_batch_ending_bucket_with_two_wave_pairs(plan_guard):
    """The CRT bucket that ends a bulk batch (plan kind 4, at least 16384
    operations) runs two p/q wave pairs per workgroup where its halves have
    8 or 16 lanes: 16384 1024-bit decryptions on an 8-lane plan (the
    16-lane one is covered by the full mixed workload), every output
    against the oracle."""
    rsagpu.set_plan(16, 4, 32, 8, 4)
    plan_guard.append((16, 4))
    p = rsagpu.get_plan(16, 4)
    assert (p.radix_bits, p.lanes_per_op) == (32, 8)
    keys = W.make_keys(1024, W.SEED_BASE + 4, 16)[:5]
    count = 16384
    bad = ops_batch_vs_oracle(keys, np.ones(count, dtype=np.int64), count, 4242)
    assert bad.size == 0, "%d of %d differ, first %d" % (bad.size, count, bad[0])
    assert rsagpu.device_errors() == 0
