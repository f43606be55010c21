"""CPU model of the radix-2^29 lane-group Montgomery product.

The GPU kernel keeps every limb position in a 64-bit accumulator and never
checks for overflow; it relies on two bounds:

* every register is drained once every L steps (its low bits move a lane
  down, the rest to the next register), so with L <= 31 limbs per lane no
  accumulator reaches 2^64 even when the inputs carry redundant limbs, and
  the product needs no normalisation inside its loop;
* lazy products (no final subtraction, redundant output limbs) keep a chain
  of products below 2n when R > 4n, so the exponentiation never compares
  with n and one canonical product at the end restores [0, n).

This model replays the kernel's position arithmetic lane by lane (the same
steps in the same order: products into rotating registers, m from lane 0,
carry of the lowest register into the next, low bits moved one lane down,
lazy or full normalisation at the end) on Python integers
and asserts both bounds at every addition, then checks the results against
Python's own modular arithmetic.  It is a check of the kernel's design, not
of the kernel: the GPU parity tests compare the kernel itself with the
oracle.
"""
import random

import pytest

MASK64 = (1 << 64) - 1


def n0inv_of(n0, B):
    # -n0^-1 mod 2^B
    return (-pow(n0, -1, 1 << B)) % (1 << B)


def to_limbs(x, S, B):
    return [(x >> (B * i)) & ((1 << B) - 1) for i in range(S)]


def value(limbs, B):
    return sum(l << (B * i) for i, l in enumerate(limbs))


class Model:
    def __init__(self, S, G, B=29):
        assert S % G == 0
        self.S, self.G, self.B, self.L = S, G, B, S // G
        self.M = (1 << B) - 1
        self.max_acc = 0

    def _add(self, acc, g, r, v):
        acc[g][r] += v
        self.max_acc = max(self.max_acc, acc[g][r])
        assert acc[g][r] <= MASK64, "accumulator overflow"

    def _lazy(self, acc):
        G, L, B, M = self.G, self.L, self.B, self.M
        his = [[a >> B for a in acc[g]] for g in range(G)]
        v = [[0] * L for _ in range(G)]
        for g in range(G):
            v[g][0] = (acc[g][0] & M) + (his[g - 1][L - 1] if g > 0 else 0)
            for j in range(1, L):
                v[g][j] = (acc[g][j] & M) + his[g][j - 1]
        # nothing may leave the group's top lane
        assert his[G - 1][L - 1] == 0
        h2 = [[x >> B for x in v[g]] for g in range(G)]
        assert h2[G - 1][L - 1] == 0
        w = []
        for g in range(G):
            w.append((v[g][0] & M) + (h2[g - 1][L - 1] if g > 0 else 0))
            for j in range(1, L):
                w.append((v[g][j] & M) + h2[g][j - 1])
        return w

    def mont_mul(self, a, b, n, lazy=True):
        """a, b, n: S limbs each (a, b possibly redundant).  Returns limbs."""
        S, G, L, B = self.S, self.G, self.L, self.B
        acc = self.product_loop(a, b, n)
        if lazy:
            return self._lazy(acc)
        # full normalisation and one conditional subtraction
        v = sum(acc[g][j] << (B * (g * L + j)) for g in range(G) for j in range(L))
        nv = value(n, B)
        if v >= nv:
            v -= nv
        assert v < nv
        return to_limbs(v, S, B)

    def product_loop(self, a, b, n):
        """The S steps of the product; returns the accumulators [lane][register]."""
        S, G, L, B, M = self.S, self.G, self.L, self.B, self.M
        ninv = n0inv_of(n[0], B)
        acc = [[0] * L for _ in range(G)]
        for i0 in range(0, S, L):
            for k in range(L):
                bi = b[i0 + k]
                for g in range(G):
                    for j in range(L):
                        self._add(acc, g, (j + k) % L, a[g * L + j] * bi)
                p0, p1 = k % L, (k + 1) % L
                m = (((acc[0][p0] & 0xFFFFFFFF) * ninv) & 0xFFFFFFFF) & M
                for g in range(G):
                    for j in range(L):
                        self._add(acc, g, (j + k) % L, m * n[g * L + j])
                for g in range(G):
                    self._add(acc, g, p1, acc[g][p0] >> B)
                low = [acc[g][p0] & M for g in range(G)]
                assert low[0] == 0, "lowest position not cleared by m*n"
                for g in range(G):
                    acc[g][p0] = low[g + 1] if g + 1 < G else low[0]
        return acc


def ubfe(x, off, wid):
    """The 32-bit unsigned bit-field extract of the AMD ISA (v_bfe_u32):
    offset and width use their low five bits."""
    return (x >> (off & 31)) & ((1 << (wid & 31)) - 1)


def sqr_loop(md, a, n):
    """The symmetric squaring's S steps (rmont_sqr_regs): step k of block q
    runs registers j >= k only; j > k multiply by 2a[qL+k] in every lane,
    j == k squares lane q's own limb, doubles the pair in lanes above q and
    adds nothing in lanes below q -- the kernel takes that multiplier out of
    the doubled limb with one bit-field extract (offset 1 in lane q, width 31
    from lane q up, width 0 below).  Returns (accumulators, multiplier slots
    run per lane)."""
    S, G, L, B, M = md.S, md.G, md.L, md.B, md.M
    ninv = n0inv_of(n[0], B)
    acc = [[0] * L for _ in range(G)]
    slots = 0
    for q in range(G):
        for k in range(L):
            b = a[q * L + k]
            b2 = 2 * b
            assert b2 < 1 << 31, "doubled limb must fit the extract's 31-bit width"
            for j in range(k, L):
                slots += 1
                for g in range(G):
                    if j > k:
                        f = b2
                    else:
                        f = ubfe(b2, 1 if g == q else 0, 31 if g >= q else 0)
                        # what the extract must give: lane q's own limb, the doubled pair, or nothing
                        assert f == (a[g * L + j] if g == q else (b2 if g > q else 0))
                    md._add(acc, g, (j + k) % L, a[g * L + j] * f)
            p0, p1 = k % L, (k + 1) % L
            m = (((acc[0][p0] & 0xFFFFFFFF) * ninv) & 0xFFFFFFFF) & M
            for g in range(G):
                for j in range(L):
                    md._add(acc, g, (j + k) % L, m * n[g * L + j])
            for g in range(G):
                md._add(acc, g, p1, acc[g][p0] >> B)
            low = [acc[g][p0] & M for g in range(G)]
            assert low[0] == 0, "lowest position not cleared by m*n"
            for g in range(G):
                acc[g][p0] = low[g + 1] if g + 1 < G else low[0]
    return acc, slots


def rand_modulus(rng, bits):
    return rng.getrandbits(bits) | (1 << (bits - 1)) | (1 << (bits - 2)) | 1


@pytest.mark.parametrize("S,G,bits", [(18, 2, 512), (36, 4, 1024), (36, 2, 1024), (28, 4, 768)])
def test_lazy_chain_matches_python(S, G, bits):
    """A chain of lazy products (squarings and products with a window table,
    as in the exponentiation) stays below 2n with bounded limbs and no
    accumulator overflow; one canonical product at the end gives x^e mod n."""
    rng = random.Random(S * 1000 + G + bits)
    B = 29
    md = Model(S, G, B)
    R = 1 << (B * S)
    for _ in range(2):
        n = rand_modulus(rng, bits)
        nl = to_limbs(n, S, B)
        x = rng.randrange(n)
        xt = to_limbs(x * R % n, S, B)
        w = 3
        table = [None, xt]
        for i in range(2, 1 << w):
            table.append(md.mont_mul(table[-1], xt, nl))
        e = rng.getrandbits(48) | (1 << 47)
        digits = []
        t = e
        while t:
            digits.append(t & ((1 << w) - 1))
            t >>= w
        A = table[digits[-1]]
        for d in reversed(digits[:-1]):
            for _ in range(w):
                A = md.mont_mul(A, A, nl)
                assert value(A, B) < 2 * n
                assert max(A) < (1 << B) + (1 << (64 - 2 * B))
            if d:
                A = md.mont_mul(A, table[d], nl)
                assert value(A, B) < 2 * n
        one = [1] + [0] * (S - 1)
        out = md.mont_mul(A, one, nl, lazy=False)
        assert value(out, B) == pow(x, e, n)


@pytest.mark.parametrize("S,G", [(18, 2), (36, 2), (36, 4), (56, 4), (72, 4), (72, 8), (144, 8), (144, 16)])
def test_accumulator_bound_with_extreme_limbs(S, G):
    """Largest limbs a lazy product can hand on (2^29 + 63) with the largest
    modulus limbs: draining every register once per L steps keeps every
    accumulator below 2^64 with no normalisation inside the product (the
    bound depends on limb sizes only, so this is the worst case)."""
    B = 29
    md = Model(S, G, B)
    big = (1 << B) + (1 << (64 - 2 * B)) - 1
    a = [big] * S
    n = [(1 << B) - 1] * S
    # synthetic inputs whose value exceeds 2^(B*S): only the product loop
    # (every addition asserts the 64-bit bound)
    md.product_loop(a, a, n)
    assert md.max_acc < (1 << 64)
    assert md.max_acc > (1 << 61)   # within a factor 8 of the limit: the check is meaningful


def test_lazy_output_bound_is_tight_enough():
    """Redundant output limbs stay below 2^29 + 2^6 over many random lazy
    products with inputs close to 2n."""
    rng = random.Random(7)
    B, S, G = 29, 18, 2
    md = Model(S, G, B)
    for _ in range(20):
        n = rand_modulus(rng, 512)
        nl = to_limbs(n, S, B)
        a = to_limbs(2 * n - 1 - rng.randrange(1000), S, B)
        b = to_limbs(2 * n - 1 - rng.randrange(1000), S, B)
        r = md.mont_mul(a, b, nl)
        R = 1 << (B * S)
        assert value(r, B) % n == value(a, B) * value(b, B) * pow(R, -1, n) % n
        assert value(r, B) < 2 * n
        assert max(r) < (1 << B) + (1 << 6)


SQR_SHAPES = [(18, 2), (28, 4), (36, 2), (36, 4), (56, 4), (72, 4)]


@pytest.mark.parametrize("S,G", SQR_SHAPES)
def test_symmetric_square_equals_general_product(S, G):
    """Each unordered pair of limbs once, doubled: the same m at every step
    (every column is complete at its drain), so the same value as the
    general product with b = a, with S*(L+1)/2 multiplier slots per lane
    instead of S*L, and the same lazy output bounds."""
    B = 29
    rng = random.Random(S * 7 + G)
    md = Model(S, G, B)
    L = S // G
    R = 1 << (B * S)
    for _ in range(4):
        n = rand_modulus(rng, B * S - 12)
        nl = to_limbs(n, S, B)
        a = to_limbs(2 * n - 1 - rng.randrange(1 << 20), S, B)
        a[1] += 1 << 6          # a redundant limb: same value, limb above 2^B
        a[2] -= 1
        acc, slots = sqr_loop(md, a, nl)
        assert slots == S * (L + 1) // 2
        w = md._lazy(acc)
        ref = md._lazy(md.product_loop(a, a, nl))
        assert value(w, B) == value(ref, B)
        assert value(w, B) % n == value(a, B) ** 2 * pow(R, -1, n) % n
        assert value(w, B) < 2 * n and max(w) < (1 << B) + (1 << 6)


@pytest.mark.parametrize("S,G", SQR_SHAPES)
def test_symmetric_square_accumulator_bound(S, G):
    """Doubled products with the largest redundant limbs: no accumulator
    reaches 2^64 for the limbs per lane the kernels square with."""
    B = 29
    md = Model(S, G, B)
    big = (1 << B) + (1 << (64 - 2 * B)) - 1
    sqr_loop(md, [big] * S, [(1 << B) - 1] * S)
    assert (1 << 61) < md.max_acc < (1 << 64)
    # the kernel's static bound (rsqr_fits) admits these shapes
    assert 3 * (S // G) <= (1 << (64 - 2 * B)) - 2
