"""Seeded synthetic RSA workloads: keys and messages.

This module only *generates inputs*.  It is shared by the test-suite, the
benchmark and the serving demo, and it holds none of the exponentiation
arithmetic that the GPU library or the CPU oracle implement: primality tests
and modular inverses use Python's built-in three-argument ``pow``.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), which is counter-based:
output i of a stream seeded with s is mix(s + (i + 1) * gamma), so whole
blocks of a stream can be drawn with numpy at once.

Key generation follows the paper's Section 3.1: two distinct random primes p
and q of equal size, n = p*q, phi(n) = (p-1)(q-1), an exponent e coprime to
phi(n), and d with d*e = 1 mod phi(n).  Readings where the paper says nothing:
each prime has its two top bits set (so n has exactly the requested number of
bits), p > q, and the CRT values dp = d mod (p-1), dq = d mod (q-1),
qinv = q^-1 mod p are kept for Chinese-remainder decryption.
"""
from __future__ import annotations

import json
import math
import os
import sys
from dataclasses import dataclass, asdict
from typing import Dict, List, Optional, Sequence

import numpy as np

MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15

# Per-workload base seeds: 14071465 + workload number.
SEED_BASE = 14071465


# ---------------------------------------------------------------------------
# SplitMix64
# ---------------------------------------------------------------------------

def _mix64(z: int) -> int:
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 & MASK64
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB & MASK64
    return z ^ (z >> 31)


def derive_seed(seed: int, *tags: int) -> int:
    """A sub-stream seed from a parent seed and integer tags."""
    s = seed & MASK64
    for t in tags:
        s = _mix64((s ^ _mix64((t + _GAMMA) & MASK64)) & MASK64)
    return s


def splitmix64_block(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream seeded with seed."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & MASK64) + idx * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


class SplitMix64:
    """Sequential SplitMix64 stream for scalar draws."""

    def __init__(self, seed: int):
        self.seed = seed & MASK64
        self.i = 0

    def next64(self) -> int:
        self.i += 1
        return _mix64((self.seed + self.i * _GAMMA) & MASK64)

    def bits(self, nbits: int) -> int:
        v, have = 0, 0
        while have < nbits:
            v |= self.next64() << have
            have += 64
        return v & ((1 << nbits) - 1)

    def below(self, bound: int) -> int:
        """Uniform integer in [0, bound) by rejection."""
        if bound <= 0:
            raise ValueError("bound must be positive")
        nb = max(1, (bound - 1).bit_length())
        while True:
            v = self.bits(nb)
            if v < bound:
                return v


# ---------------------------------------------------------------------------
# primes and keys
# ---------------------------------------------------------------------------

def _small_primes(limit: int) -> List[int]:
    sieve = bytearray([1]) * limit
    sieve[0:2] = b"\x00\x00"
    for i in range(2, int(limit ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = bytearray(len(sieve[i * i::i]))
    return [i for i in range(limit) if sieve[i]]


_SMALL = _small_primes(2000)
_PRIMORIAL = math.prod(_SMALL)
_DETERMINISTIC_BASES = _SMALL[:13]      # exact for every n < 3.3e24


def is_probable_prime(c: int, rng: SplitMix64, rounds: int) -> bool:
    """Miller-Rabin.  Below 2^80 the first 13 prime bases make it exact;
    above, ``rounds`` random bases in [2, c-2] are drawn from ``rng``."""
    if c < 2:
        return False
    for p in _SMALL[:40]:
        if c == p:
            return True
        if c % p == 0:
            return False
    d, r = c - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    if c.bit_length() <= 80:
        bases = _DETERMINISTIC_BASES
    else:
        bases = [2 + rng.below(c - 3) for _ in range(rounds)]
    for a in bases:
        x = pow(a, d, c)
        if x == 1 or x == c - 1:
            continue
        for _ in range(r - 1):
            x = x * x % c
            if x == c - 1:
                break
        else:
            return False
    return True


def mr_rounds(bits: int) -> int:
    """Random-base Miller-Rabin rounds for a random prime candidate."""
    return 40 if bits < 512 else 24


def random_prime(bits: int, rng: SplitMix64, e: int) -> int:
    """A random prime of exactly ``bits`` bits with its two top bits set and
    gcd(e, p-1) = 1."""
    if bits < 3:
        raise ValueError("prime too small")
    top = 3 << (bits - 2)
    while True:
        c = rng.bits(bits) | top | 1
        if c > _SMALL[-1] and math.gcd(c, _PRIMORIAL) != 1:
            continue
        if math.gcd(e, c - 1) != 1:
            continue
        if is_probable_prime(c, rng, mr_rounds(bits)):
            return c


@dataclass(frozen=True)
class RSAKey:
    bits: int
    n: int
    e: int
    d: int
    p: int
    q: int
    dp: int
    dq: int
    qinv: int

    @property
    def limbs(self) -> int:
        return (self.bits + 31) // 32

    def check(self) -> None:
        """Consistency of the key (raises AssertionError)."""
        phi = (self.p - 1) * (self.q - 1)
        assert self.p > self.q > 1 and self.n == self.p * self.q
        assert self.n.bit_length() == self.bits
        assert (self.e * self.d) % phi == 1 and 1 < self.e < phi
        assert self.dp == self.d % (self.p - 1) and self.dq == self.d % (self.q - 1)
        assert (self.qinv * self.q) % self.p == 1 and 0 < self.qinv < self.p


def make_key(bits: int, seed: int, e: int = 65537) -> RSAKey:
    """Seeded RSA key with a ``bits``-bit modulus (Section 3.1)."""
    if bits % 2:
        raise ValueError("modulus bits must be even")
    rng = SplitMix64(seed)
    half = bits // 2
    p = random_prime(half, rng, e)
    while True:
        q = random_prime(half, rng, e)
        if q != p:
            break
    if p < q:
        p, q = q, p
    n = p * q
    phi = (p - 1) * (q - 1)
    d = pow(e, -1, phi)
    key = RSAKey(bits, n, e, d, p, q, d % (p - 1), d % (q - 1), pow(q, -1, p))
    key.check()
    return key


def _cache_dir() -> str:
    here = os.path.dirname(os.path.abspath(__file__))
    return os.environ.get("RSAGPU_KEY_CACHE", os.path.join(os.path.dirname(here), ".keycache"))


def _make_key_args(args):
    return make_key(*args)


def make_keys(bits: int, seed: int, count: int, e: int = 65537,
              processes: Optional[int] = None, cache: bool = True) -> List[RSAKey]:
    """``count`` keys; key j is make_key(bits, derive_seed(seed, bits, j), e).

    Keys are cached as JSON under ``.keycache/`` beside the package (checked
    again on load) and generated with a process pool when missing."""
    path = os.path.join(_cache_dir(), "keys_%d_%d_%d_%d.json" % (bits, seed, count, e))
    if cache and os.path.exists(path):
        try:
            with open(path) as f:
                raw = json.load(f)
            keys = [RSAKey(**{k: int(v, 16) if isinstance(v, str) else v for k, v in r.items()})
                    for r in raw]
            for k in keys:
                k.check()
            if len(keys) == count:
                return keys
        except (OSError, ValueError, AssertionError, TypeError):
            pass
    args = [(bits, derive_seed(seed, bits, j), e) for j in range(count)]
    if processes is None:
        processes = min(count, 16, os.cpu_count() or 1)
    # no worker processes once this process has initialised a GPU
    tmod = sys.modules.get("torch")
    if tmod is not None and getattr(tmod, "cuda", None) is not None and tmod.cuda.is_initialized():
        processes = 1
    if processes > 1 and count > 1 and bits >= 512:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(processes) as pool:
            keys = pool.map(_make_key_args, args)
    else:
        keys = [make_key(*a) for a in args]
    if cache:
        try:
            os.makedirs(_cache_dir(), exist_ok=True)
            tmp = path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump([{k: (hex(v) if k not in ("bits", "e") else v)
                            for k, v in asdict(key).items()} for key in keys], f)
            os.replace(tmp, path)
        except OSError:
            pass
    return keys


# ---------------------------------------------------------------------------
# limb arrays
# ---------------------------------------------------------------------------

def ints_to_limbs(values: Sequence[int], limbs: int) -> np.ndarray:
    """(count, limbs) uint32, little-endian limbs, message-major."""
    nbytes = 4 * limbs
    buf = b"".join(int(v).to_bytes(nbytes, "little") for v in values)
    return np.frombuffer(buf, dtype="<u4").reshape(len(values), limbs).astype(np.uint32)


def limbs_to_ints(arr: np.ndarray) -> List[int]:
    arr = np.ascontiguousarray(arr, dtype="<u4")
    if arr.ndim == 1:
        arr = arr[None, :]
    return [int.from_bytes(row.tobytes(), "little") for row in arr]


def int_to_limbs(value: int, limbs: int) -> np.ndarray:
    return ints_to_limbs([value], limbs)[0]


def uniform_below(n: int, count: int, seed: int, limbs: Optional[int] = None) -> np.ndarray:
    """``count`` integers uniform in [0, n) as a (count, limbs) uint32 array.

    Rows of bitlen(n) random bits are drawn from the stream in order and those
    >= n are rejected, so the result depends only on (n, count, seed)."""
    L = limbs or (n.bit_length() + 31) // 32
    nb = n.bit_length()
    words = (L + 1) // 2
    nl = int_to_limbs(n, L)
    top = (nb - 1) // 32                       # limb holding the top bit of n
    top_mask = np.uint32((1 << (nb - 32 * top)) - 1)
    out = []
    got, start = 0, 0
    while got < count:
        want = max(64, int((count - got) * 1.25) + 16)
        raw = splitmix64_block(seed, start, want * words)
        start += want * words
        rows = raw.view(np.uint32).reshape(want, 2 * words)[:, :L].copy()
        rows[:, top] &= top_mask
        rows[:, top + 1:] = 0
        # rows < n, compared lexicographically from the top limb
        diff = rows != nl
        anyd = diff.any(axis=1)
        topd = L - 1 - np.argmax(diff[:, ::-1], axis=1)
        less = anyd & (rows[np.arange(want), topd] < nl[topd])
        acc = rows[less]
        out.append(acc)
        got += acc.shape[0]
    return np.concatenate(out)[:count]


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    """One synthetic workload: keys plus message and ciphertext arrays."""
    name: str
    seed: int
    keys: List[RSAKey]
    key_of: np.ndarray          # (count,) key index of every element
    msgs: np.ndarray            # (count, limbs) plaintexts in [0, n)
    ctxt: np.ndarray            # (count, limbs) ciphertexts to decrypt, in [0, n)
    limbs: int


def messages_for_keys(keys: List[RSAKey], count: int, seed: int, tag: int):
    """Element i belongs to key i mod len(keys); per-key uniform draws."""
    K = len(keys)
    L = keys[0].limbs
    key_of = np.arange(count, dtype=np.int32) % K
    out = np.zeros((count, L), dtype=np.uint32)
    for j, key in enumerate(keys):
        idx = np.nonzero(key_of == j)[0]
        if idx.size:
            out[idx] = uniform_below(key.n, idx.size, derive_seed(seed, tag, j), L)
    return key_of, out


def single_size_workload(name: str, bits: int, nkeys: int, count: int, seed: int) -> Workload:
    keys = make_keys(bits, seed, nkeys)
    key_of, msgs = messages_for_keys(keys, count, seed, 1)
    _, ctxt = messages_for_keys(keys, count, seed, 2)
    return Workload(name, seed, keys, key_of, msgs, ctxt, keys[0].limbs)


# The fixed workloads.  ``count`` may be lowered for parity tests at small size.
def workload_c1(count: int = 4096) -> Workload:
    """64-bit modulus, one key, e = 65537, full-d decryption."""
    return single_size_workload("rsa64-1key", 64, 1, count, SEED_BASE + 1)


def workload_c2(count: int = 65536) -> Workload:
    """1024-bit modulus, one key, e = 65537, full-d decryption (no CRT)."""
    return single_size_workload("rsa1024-1key", 1024, 1, count, SEED_BASE + 2)


def workload_c3(count: int = 16384, nkeys: int = 64) -> Workload:
    """2048-bit moduli, 64 keys, messages round-robin; CRT decryption."""
    return single_size_workload("rsa2048-64keys", 2048, nkeys, count, SEED_BASE + 3)


def workload_crt4096(count: int = 1092) -> Workload:
    """4096-bit moduli, the 16 keys of the mixed workload's 4096-bit class,
    messages round-robin; by default as many as that workload's 4096-bit
    CRT decryptions."""
    return single_size_workload("rsa4096-16keys", 4096, 16, count, SEED_BASE + 4)


@dataclass
class MixedWorkload:
    """Operations over keys of several sizes, laid out for rsa_ops_batch."""
    name: str
    keys: List[RSAKey]          # key id = index
    kinds: np.ndarray           # (nops,) 0 = encrypt, 1 = CRT decrypt
    key_ids: np.ndarray         # (nops,)
    in_offs: np.ndarray         # (nops,) word offsets into in_pool
    in_pool: np.ndarray         # uint32 words: op i's input at in_offs[i] (its key's limbs words)
    out_words: int              # size of the output pool (same offsets)


def largest_remainder(total: int, weights: Sequence[int]) -> List[int]:
    """Integer split of total proportional to weights (largest remainder)."""
    s = sum(weights)
    raw = [total * w / s for w in weights]
    base = [int(math.floor(r)) for r in raw]
    order = sorted(range(len(weights)), key=lambda i: raw[i] - base[i], reverse=True)
    for i in order[:total - sum(base)]:
        base[i] += 1
    return base


def mixed_workload(name: str, sizes: Sequence[int], weights: Sequence[int], total: int,
                   keys_per_size: int, seed: int) -> MixedWorkload:
    """Ops over `keys_per_size` keys of each size; within a size, even op
    index = encryption and odd = CRT decryption, keys round-robin; inputs
    uniform in [0, n); op order shuffled with a seeded permutation."""
    counts = largest_remainder(total, weights)
    keys: List[RSAKey] = []
    kinds, kids, inputs = [], [], []
    for si, (bits, cnt) in enumerate(zip(sizes, counts)):
        ks = make_keys(bits, seed, keys_per_size)
        first = len(keys)
        keys.extend(ks)
        L = ks[0].limbs
        k_of = np.arange(cnt) % keys_per_size
        vals = np.zeros((cnt, L), dtype=np.uint32)
        for j, key in enumerate(ks):
            idx = np.nonzero(k_of == j)[0]
            if idx.size:
                vals[idx] = uniform_below(key.n, idx.size, derive_seed(seed, bits, j, 3), L)
        kinds.append(np.arange(cnt) % 2)
        kids.append(first + k_of)
        inputs.extend(vals)
    kinds_a = np.concatenate(kinds).astype(np.int64)
    kids_a = np.concatenate(kids).astype(np.int64)
    perm = np.argsort(splitmix64_block(derive_seed(seed, 77), 0, len(kinds_a)), kind="stable")
    kinds_a, kids_a = kinds_a[perm], kids_a[perm]
    inputs = [inputs[i] for i in perm.tolist()]
    lens = np.array([len(v) for v in inputs], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    pool = np.concatenate(inputs).astype(np.uint32) if inputs else np.zeros(0, np.uint32)
    return MixedWorkload(name, keys, kinds_a, kids_a, offs, pool, int(lens.sum()))


def workload_c4(total: int = 32768, keys_per_size: int = 16) -> MixedWorkload:
    """1024/2048/3072/4096-bit keys in ratio 4:8:2:1, half encryptions
    (e = 65537), half CRT decryptions, 16 keys per size."""
    return mixed_workload("rsa-mixed-1k-4k", [1024, 2048, 3072, 4096], [4, 8, 2, 1], total,
                          keys_per_size, SEED_BASE + 4)


# ---------------------------------------------------------------------------
# the paper's own experiment (Section 10): one-word moduli, 8-bit exponents
# ---------------------------------------------------------------------------

@dataclass
class PaperTableKey:
    """A key of the paper's experiments: n printed in Tables 1 and 2, e an
    8-bit exponent.  Table 1 uses n = 131 * 137 with e = 131 (the example key
    of Section 2); its printed private exponent 137 does not invert e modulo
    phi(n) = 17680, so d here is the inverse, 14171.  Table 2's caption
    prints 1005 * 509 while its text prints 1009 * 509 (1005 is not prime):
    n = 513581; the paper gives no exponent for it, so it takes the same
    8-bit e = 131, which is coprime to phi(n) = 512064."""
    table: int
    p: int
    q: int
    e: int

    @property
    def n(self) -> int:
        return self.p * self.q

    @property
    def d(self) -> int:
        return pow(self.e, -1, (self.p - 1) * (self.q - 1))


PAPER_TABLE_KEYS = {1: PaperTableKey(1, 137, 131, 131), 2: PaperTableKey(2, 1009, 509, 131)}
# Data sizes of Tables 1 and 2 (the last two printed as 16392 and 32784,
# read as 16384 and 32768: blocks x threads per block).
PAPER_TABLE_SIZES = (256, 512, 1024, 2048, 4096, 8192, 16384, 32768)
# Times the tables print (units as printed, likely not seconds), by data size.
PAPER_TABLE_GPU_TIME = {
    1: (7.56, 7.25, 6.86, 5.38, 5.68, 6.27, 7.21, 9.25),
    2: (6.08, 6.52, 6.69, 5.53, 6.58, 6.66, 7.81, 8.76),
}


def paper_table_messages(count: int, seed: int = SEED_BASE + 6) -> np.ndarray:
    """``count`` messages uniform in 0..800 (the paper's test messages cover
    the ASCII table), one 32-bit limb each: (count, 1) uint32."""
    return uniform_below(801, count, seed, 1)


def text_to_packets(text: str) -> List[int]:
    """Section 2's encoding of a text: letters a..z as 00..25 (other
    characters dropped), two letters per packet as a four-digit decimal
    number (a trailing single letter pads with 'x' = 23)."""
    codes = [ord(ch) - 97 for ch in text.lower() if "a" <= ch <= "z"]
    if len(codes) % 2:
        codes.append(23)
    return [codes[i] * 100 + codes[i + 1] for i in range(0, len(codes), 2)]


def packets_to_text(packets: Sequence[int]) -> str:
    """Inverse of text_to_packets (letters only)."""
    return "".join(chr(97 + p // 100) + chr(97 + p % 100) for p in packets)
