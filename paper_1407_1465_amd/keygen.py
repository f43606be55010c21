"""Batched RSA key generation with the GPU doing the primality tests.

Section 3.1 builds a key from two random primes.  Finding a prime of b bits
means testing ~b/2 candidates (after trial division) with Miller-Rabin,
whose cost is one modular exponentiation a^d mod c per round: for 2048-bit
primes that is the wait before any 4096-bit key exists.  Here the rounds of
many candidates of many keys run as batched ``rsa_modexp_batch`` calls (the
library's hot path), and the host only draws candidates and assembles keys.

The keys are exactly those of ``workloads.make_key`` for the same seed: the
candidates and their random bases are drawn from the same SplitMix64 stream
in the same order (every candidate that reaches Miller-Rabin draws all its
bases before the first is tried, so the stream does not depend on the test
results), and p and q are the first two distinct candidates that pass.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

from . import workloads as W

Candidate = Tuple[int, List[int]]       # (candidate, Miller-Rabin bases)


def _draw_candidates(rng: W.SplitMix64, bits: int, e: int, count: int) -> List[Candidate]:
    """The next ``count`` candidates of ``random_prime``'s stream that reach
    Miller-Rabin, each with the bases ``is_probable_prime`` draws for it."""
    top = 3 << (bits - 2)
    rounds = W.mr_rounds(bits)
    out: List[Candidate] = []
    while len(out) < count:
        c = rng.bits(bits) | top | 1
        if c > W._SMALL[-1] and math.gcd(c, W._PRIMORIAL) != 1:
            continue
        if math.gcd(e, c - 1) != 1:
            continue
        if c.bit_length() <= 80:
            bases = list(W._DETERMINISTIC_BASES)
        else:
            bases = [2 + rng.below(c - 3) for _ in range(rounds)]
        out.append((c, bases))
    return out


def _trial_division(c: int):
    """is_probable_prime's trial division by the first 40 primes: True/False
    when it decides, None when Miller-Rabin must."""
    for p in W._SMALL[:40]:
        if c == p:
            return True
        if c % p == 0:
            return False
    return None


def miller_rabin_gpu(pairs: Sequence[Tuple[int, int]], limbs: int, rsagpu, torch) -> List[bool]:
    """For each (c, a): does base a let c pass one Miller-Rabin round?  With
    c - 1 = d * 2^r (d odd): a^d mod c is 1 or c - 1, or one of its next
    r - 1 squarings is c - 1.  Every exponentiation runs on the GPU."""
    if not pairs:
        return []
    cs = [c for c, _ in pairs]
    ds, rs = [], []
    for c in cs:
        d, r = c - 1, 0
        while d % 2 == 0:
            d //= 2
            r += 1
        ds.append(d)
        rs.append(r)

    def dev(vals):
        a = W.ints_to_limbs(vals, limbs)
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()

    mod = dev(cs)
    x = rsagpu.modexp(dev([a % c for c, a in pairs]), dev(ds), mod)
    xs = W.limbs_to_ints(x.cpu().numpy().view(np.uint32))
    ok = [v == 1 or v == c - 1 for v, c in zip(xs, cs)]
    todo = [i for i in range(len(cs)) if not ok[i] and rs[i] > 1]
    step = 1
    while todo:
        sel = torch.tensor(todo, dtype=torch.long, device="cuda")
        two = dev([2] * len(todo))
        x_sel = rsagpu.modexp(x[sel].contiguous(), two, mod[sel].contiguous())
        x[sel] = x_sel
        vals = W.limbs_to_ints(x_sel.cpu().numpy().view(np.uint32))
        nxt = []
        for i, v in zip(todo, vals):
            if v == cs[i] - 1:
                ok[i] = True
            elif step + 1 < rs[i]:
                nxt.append(i)
        todo = nxt
        step += 1
    return ok


def make_keys_gpu(bits: int, seed: int, count: int, e: int = 65537, chunk: int = 0) -> List[W.RSAKey]:
    """``count`` keys equal to ``workloads.make_keys(bits, seed, count, e)``,
    key j from seed derive_seed(seed, bits, j), with the Miller-Rabin rounds
    batched on the GPU across candidates and keys."""
    import torch
    from . import rsagpu
    if bits % 2:
        raise ValueError("modulus bits must be even")
    half = bits // 2
    limbs = (half + 31) // 32
    chunk = chunk or max(16, half // 16)      # candidates per key per pass (about 2 primes' worth)
    rngs = [W.SplitMix64(W.derive_seed(seed, bits, j)) for j in range(count)]
    found: List[List[int]] = [[] for _ in range(count)]
    pending = list(range(count))
    while pending:
        cands = {j: _draw_candidates(rngs[j], half, e, chunk) for j in pending}
        # first round for every candidate, the remaining rounds for those that pass it
        first = [(j, k) for j in pending for k in range(len(cands[j]))]
        passed = {}
        need_mr = []
        for j, k in first:
            c = cands[j][k][0]
            v = _trial_division(c)
            if v is None:
                need_mr.append((j, k))
            else:
                passed[(j, k)] = v
        r1 = miller_rabin_gpu([(cands[j][k][0], cands[j][k][1][0]) for j, k in need_mr], limbs, rsagpu, torch)
        rest = []
        for (j, k), ok in zip(need_mr, r1):
            if ok:
                rest.extend(((j, k), a) for a in cands[j][k][1][1:])
            passed[(j, k)] = ok
        r2 = miller_rabin_gpu([(cands[j][k][0], a) for (j, k), a in rest], limbs, rsagpu, torch)
        for ((j, k), _), ok in zip(rest, r2):
            passed[(j, k)] = passed[(j, k)] and ok
        still = []
        for j in pending:
            for k in range(len(cands[j])):
                c = cands[j][k][0]
                if len(found[j]) < 2 and passed[(j, k)] and c not in found[j]:
                    found[j].append(c)
            if len(found[j]) < 2:
                still.append(j)
        pending = still
    keys = []
    for j in range(count):
        p, q = found[j]
        if p < q:
            p, q = q, p
        n = p * q
        phi = (p - 1) * (q - 1)
        d = pow(e, -1, phi)
        key = W.RSAKey(bits, n, e, d, p, q, d % (p - 1), d % (q - 1), pow(q, -1, p))
        key.check()
        keys.append(key)
    return keys
