"""Resident keys and mixed batches (rsa_keyset_*, rsa_ops_batch) against the
CPU oracle, bit-exact; invalid descriptors; alone-versus-mixed equality."""
import random

import numpy as np
import pytest

from paper_1407_1465_amd import workloads as W
from gpu_util import dev, host, oracle_modexp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_1465_amd import rsagpu  # noqa: E402


def make_keyset(keys):
    ks = rsagpu.KeySet(len(keys) + 4)
    for k in keys:
        ks.add(k.limbs, k.n, k.e, k.p, k.q, k.dp, k.dq, k.qinv)
    return ks


def run_ops(ks, kinds, key_ids, in_offs, in_pool, out_words, out_offs=None):
    out_offs = in_offs if out_offs is None else out_offs
    ops = rsagpu.pack_ops(kinds, key_ids, in_offs, out_offs).cuda()
    inp = dev(in_pool)
    out = torch.zeros(out_words, dtype=torch.int32, device="cuda")
    ws = torch.empty(rsagpu.ops_workspace_size(len(kinds)), dtype=torch.uint8, device="cuda")
    rsagpu.ops_batch(ks, ops, inp, out, ws)
    return host(out)


def oracle_ops(keys, kinds, key_ids, in_offs, in_pool):
    """Expected output words per op: in^e or in^d mod n (plain, no CRT)."""
    res = []
    by_width = {}
    for i, (kd, kid, off) in enumerate(zip(kinds, key_ids, in_offs)):
        k = keys[kid]
        by_width.setdefault(k.limbs, []).append((i, kd, k, off))
    for L, items in by_width.items():
        base = np.stack([in_pool[off:off + L] for _, _, _, off in items])
        exps = W.ints_to_limbs([k.e if kd == 0 else k.d for _, kd, k, _ in items], L)
        mods = W.ints_to_limbs([k.n for _, _, k, _ in items], L)
        out = oracle_modexp(base, exps, mods)
        res.extend((i, out[j]) for j, (i, _, _, _) in enumerate(items))
    return dict(res)


def small_mix(seed, sizes=(64, 256, 512, 1024, 2048), per_size=2, count=150):
    keys = []
    for bits in sizes:
        keys.extend(W.make_keys(bits, 900 + bits, per_size))
    rng = random.Random(seed)
    kinds, kids, offs, pool = [], [], [], []
    off = 0
    for i in range(count):
        kid = rng.randrange(len(keys))
        k = keys[kid]
        v = rng.randrange(k.n)
        if i % 17 == 0:
            v = 0
        elif i % 19 == 0:
            v = k.n - 1
        kinds.append(i % 2)
        kids.append(kid)
        offs.append(off)
        pool.extend(W.int_to_limbs(v, k.limbs).tolist())
        off += k.limbs
    return keys, np.array(kinds), np.array(kids), np.array(offs), np.array(pool, dtype=np.uint32), off


def test_keyset_mixed_vs_oracle():
    keys, kinds, kids, offs, pool, words = small_mix(1)
    ks = make_keyset(keys)
    out = run_ops(ks, kinds, kids, offs, pool, words)
    want = oracle_ops(keys, kinds, kids, offs, pool)
    for i in range(len(kinds)):
        L = keys[kids[i]].limbs
        assert np.array_equal(out[offs[i]:offs[i] + L], want[i]), "op %d (kind %d, %d bits)" % (
            i, kinds[i], 32 * L)
    assert rsagpu.device_errors() == 0
    ks.close()


@pytest.mark.parametrize("crt_runs,encs", [
    ([3] * 12, 4),          # 12 keys' runs rounded up to whole waves exceed the list: runs back to back
    ([5, 33, 1], 160),      # the rounded runs fit: each key's run starts a wave, the gaps hold empty slots
])
def test_ops_batch_crt_key_runs(crt_runs, encs):
    """A CRT bucket whose per-key runs are not whole waves, shuffled among
    encryptions of the same keys: every output equals the oracle's, whether
    the bucket list holds the runs padded to whole waves or back to back."""
    keys = W.make_keys(512, 5120 + len(crt_runs), len(crt_runs))
    rng = random.Random(len(crt_runs))
    descs = [(1, k) for k, n in enumerate(crt_runs) for _ in range(n)]
    descs += [(0, rng.randrange(len(keys))) for _ in range(encs)]
    rng.shuffle(descs)
    kinds, kids, offs, pool = [], [], [], []
    off = 0
    for kd, kid in descs:
        k = keys[kid]
        kinds.append(kd)
        kids.append(kid)
        offs.append(off)
        pool.extend(W.int_to_limbs(rng.randrange(k.n), k.limbs).tolist())
        off += k.limbs
    kinds, kids, offs = np.array(kinds), np.array(kids), np.array(offs)
    pool = np.array(pool, dtype=np.uint32)
    ks = make_keyset(keys)
    out = run_ops(ks, kinds, kids, offs, pool, off)
    want = oracle_ops(keys, kinds, kids, offs, pool)
    L = keys[0].limbs
    for i in range(len(kinds)):
        assert np.array_equal(out[offs[i]:offs[i] + L], want[i]), "op %d (kind %d)" % (i, kinds[i])
    assert rsagpu.device_errors() == 0
    ks.close()


@pytest.mark.parametrize("window", [0, 6])
def test_bulk_batch_crt_bucket_pairs_and_fallback(window):
    """In a bulk batch (at least 16384 operations) every CRT bucket runs two
    wave pairs per workgroup where the LDS holds them: 16128 512-bit CRT
    decryptions beside 256 operations of a wider key (so the 512-bit bucket
    takes the kind-3 plan), on the default plan (two pairs fit) and on a
    6-bit window whose tables fit one pair only (the bucket falls back to
    one); every output against the oracle."""
    small = W.make_keys(512, 5150, 3)
    keys = small + W.make_keys(1024, W.SEED_BASE + 4, 16)[:1]
    lds_limit = 160 * 1024
    if window:
        rsagpu.set_plan(8, 3, 32, 1, window)
    try:
        lds = rsagpu.get_plan(8, 3).lds_bytes
        assert (4 * lds + 16 <= lds_limit) == (window == 0)
        rng = random.Random(window + 11)
        descs = [(1, i % 3) for i in range(16128)] + [(i % 2, 3) for i in range(256)]
        rng.shuffle(descs)
        kinds, kids, offs, pool = [], [], [], []
        off = 0
        for kd, kid in descs:
            k = keys[kid]
            kinds.append(kd)
            kids.append(kid)
            offs.append(off)
            pool.extend(W.int_to_limbs(rng.randrange(k.n), k.limbs).tolist())
            off += k.limbs
        kinds, kids, offs = np.array(kinds), np.array(kids), np.array(offs)
        pool = np.array(pool, dtype=np.uint32)
        ks = make_keyset(keys)
        out = run_ops(ks, kinds, kids, offs, pool, off)
        want = oracle_ops(keys, kinds, kids, offs, pool)
        bad = [i for i in range(len(kinds))
               if not np.array_equal(out[offs[i]:offs[i] + keys[kids[i]].limbs], want[i])]
        assert not bad, "%d of %d differ, first %d" % (len(bad), len(kinds), bad[0])
        assert rsagpu.device_errors() == 0
        ks.close()
    finally:
        if window:
            rsagpu.set_plan(8, 3, 0, 0, 0)


def test_keyset_sixteen_lane_plans_vs_oracle():
    """Ops-batch plans on the 16-lane instances whose limb count is not the
    keyset's (S = 80 for 2048-bit operands, 64 for 1536-bit): the kernels
    compute their Montgomery constants themselves; 4096- and 3072-bit CRT
    halves and 2048-bit encryptions against the oracle."""
    touched = [(64, 3), (48, 3), (64, 2)]
    try:
        rsagpu.set_plan(64, 3, 29, 16, 4)
        rsagpu.set_plan(48, 3, 29, 16, 4)
        rsagpu.set_plan(64, 2, 29, 16, 3)
        assert rsagpu.get_plan(64, 3).padded_limbs == 80
        assert rsagpu.get_plan(48, 3).padded_limbs == 64
        keys, kinds, kids, offs, pool, words = small_mix(5, sizes=(2048, 3072, 4096), per_size=2, count=40)
        ks = make_keyset(keys)
        out = run_ops(ks, kinds, kids, offs, pool, words)
        want = oracle_ops(keys, kinds, kids, offs, pool)
        for i in range(len(kinds)):
            L = keys[kids[i]].limbs
            assert np.array_equal(out[offs[i]:offs[i] + L], want[i]), "op %d (kind %d, %d bits)" % (
                i, kinds[i], 32 * L)
        assert rsagpu.device_errors() == 0
        ks.close()
    finally:
        for limbs, kind in touched:
            rsagpu.set_plan(limbs, kind, 0, 0, 0)


def test_alone_equals_mixed():
    """Each request's result is the same alone and inside a busy mix."""
    keys, kinds, kids, offs, pool, words = small_mix(2, count=120)
    ks = make_keyset(keys)
    mixed = run_ops(ks, kinds, kids, offs, pool, words)
    for i in (0, 1, 7, 50, 119):
        L = keys[kids[i]].limbs
        alone = run_ops(ks, kinds[i:i + 1], kids[i:i + 1], np.array([0]),
                        pool[offs[i]:offs[i] + L], L)
        assert np.array_equal(alone, mixed[offs[i]:offs[i] + L])
    assert rsagpu.device_errors() == 0
    ks.close()


def test_invalid_ops_are_skipped_and_counted():
    keys, kinds, kids, offs, pool, words = small_mix(3, count=20)
    ks = make_keyset(keys)
    kids = kids.copy()
    kinds = kinds.copy()
    offs = offs.copy()
    kids[3] = 999                      # unknown key
    kinds[5] = 7                       # unknown kind
    offs[8] = words                    # input range past the pool
    out = run_ops(ks, kinds, kids, offs, pool, words + 64, out_offs=offs)
    assert rsagpu.device_errors() == 3
    want = oracle_ops(keys, kinds, np.where(kids == 999, 0, kids), offs, np.concatenate([pool, np.zeros(64, np.uint32)]))
    for i in range(len(kinds)):
        if i in (3, 5, 8):
            continue
        L = keys[kids[i]].limbs
        assert np.array_equal(out[offs[i]:offs[i] + L], want[i])
    ks.close()


def test_keyset_rejects_bad_keys():
    k = W.make_key(256, 55)
    ks = rsagpu.KeySet(4)
    with pytest.raises(rsagpu.RSAError):
        ks.add(k.limbs, k.n, k.e, k.q, k.p, k.dq, k.dp, k.qinv)           # p < q
    with pytest.raises(rsagpu.RSAError):
        ks.add(k.limbs, k.n + 2, k.e, k.p, k.q, k.dp, k.dq, k.qinv)       # n != p q
    with pytest.raises(rsagpu.RSAError):
        ks.add(k.limbs, k.n, 0, k.p, k.q, k.dp, k.dq, k.qinv)             # e = 0
    assert ks.add(k.limbs, k.n, k.e, k.p, k.q, k.dp, k.dq, k.qinv) == 0
    ks.close()


def test_workload_mixed_sizes_full():
    """32768 ops over 1024/2048/3072/4096-bit keys (4:8:2:1) in one bulk
    rsa_ops_batch call: every output against the oracle, and the whole batch
    through the round trip."""
    w = W.workload_c4()
    ks = make_keyset(w.keys)
    out = run_ops(ks, w.kinds, w.key_ids, w.in_offs, w.in_pool, w.out_words)
    assert rsagpu.device_errors() == 0
    want = oracle_ops(w.keys, w.kinds, w.key_ids, w.in_offs, w.in_pool)
    bad = [i for i in range(len(w.kinds))
           if not np.array_equal(out[w.in_offs[i]:w.in_offs[i] + w.keys[w.key_ids[i]].limbs], want[i])]
    assert not bad, "%d of %d operations differ, first %d" % (len(bad), len(w.kinds), bad[0])
    # round trip: apply the opposite operation to every output
    back = run_ops(ks, 1 - w.kinds, w.key_ids, w.in_offs, out, w.out_words)
    assert np.array_equal(back, w.in_pool)
    assert rsagpu.device_errors() == 0
    ks.close()
