// Lane-group multi-precision arithmetic in radix 2^B, B < 32 (reduced radix).
//
// Same lane-group layout as group_bn.hpp (G lanes per integer, L = S / G limbs
// per lane), but every limb holds B < 32 bits in a 32-bit word.  A product of
// two limbs is below 2^(2B), so a 64-bit accumulator absorbs 2^(64 - 2B)
// products without overflow: the Montgomery loop is one v_mad_u64_u32 per
// product with no carry detection at all.  For B = 29 that is 64 products.
// The CIOS loop adds two products per register per step, and every register
// is drained once every L steps (when it holds the lane's lowest position, its
// low B bits move one lane down and the rest, below 2^(64-B), moves to the
// next register), so a register never holds more than 2L products plus two
// small terms: L <= 31 limbs per lane keeps every accumulator below 2^64 with
// no normalisation inside the product.
//
// Integers enter and leave in the caller's 32-bit-limb format; conversion
// happens at load time (each lane reads the 32-bit words that hold its limbs)
// and at store time (through LDS, since an output word can straddle lanes).
#pragma once

#include "group_bn.hpp"

namespace rsagpu {

template <int B>
struct Radix {
    static_assert(B >= 24 && B <= 30, "reduced radix");
    static constexpr uint32_t MASK = (1u << B) - 1u;
};

// ---- conversion ------------------------------------------------------------

// Limbs [r*L, r*L + L) of the B-bit-limb form of (number at p >> bitoff),
// where the number has nwords 32-bit words (zero beyond; zero when !live).
template <int S, int G, int B>
__device__ __forceinline__ void rload(uint32_t (&x)[S / G], const uint32_t *p, int nwords, int bitoff, bool live)
{
    constexpr int L = S / G;
    const int r = grp_lane<G>();
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const int pos = bitoff + B * (r * L + k);
        const int w = pos >> 5, sh = pos & 31;
        const uint32_t lo = (live && w < nwords) ? p[w] : 0u;
        const uint32_t hi = (live && w + 1 < nwords) ? p[w + 1] : 0u;
        const uint64_t v = (((uint64_t)hi << 32) | lo) >> sh;
        x[k] = (uint32_t)v & Radix<B>::MASK;
    }
}

// Word k (32 bits) of an integer held as `nlimbs` B-bit limbs at q[0 ..].
template <int B>
__device__ __forceinline__ uint32_t rword(const uint32_t *q, int nlimbs, int k)
{
    const int pos = 32 * k;
    const int j = pos / B, sh = pos % B;
    const uint64_t l0 = j < nlimbs ? q[j] : 0u;
    const uint64_t l1 = j + 1 < nlimbs ? q[j + 1] : 0u;
    const uint64_t l2 = j + 2 < nlimbs ? q[j + 2] : 0u;
    const uint64_t v = (l0 | (l1 << B)) >> sh;
    return (uint32_t)(v | (l2 << (2 * B - sh)));
}

// ---- group-wide add / subtract / compare ---------------------------------

template <int S, int G, int B>
__device__ __forceinline__ uint32_t rgrp_add(uint32_t (&x)[S / G], const uint32_t (&y)[S / G])
{
    constexpr int L = S / G;
    constexpr uint32_t M = Radix<B>::MASK;
    uint32_t c = 0;
    bool all = true;
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const uint32_t t = x[j] + y[j] + c;
        x[j] = t & M;
        c = t >> B;
        all = all && x[j] == M;
    }
    uint32_t k = grp_carry_in<G>(c != 0, all);
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const uint32_t t = x[j] + k;
        x[j] = t & M;
        k = t >> B;
    }
    return grp_top_flag<G>((c | k) != 0) ? 1u : 0u;
}

template <int S, int G, int B>
__device__ __forceinline__ uint32_t rgrp_sub(uint32_t (&d)[S / G], const uint32_t (&x)[S / G],
                                             const uint32_t (&y)[S / G])
{
    constexpr int L = S / G;
    constexpr uint32_t M = Radix<B>::MASK;
    uint32_t b = 0, any = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const uint32_t t = x[j] - y[j] - b;
        d[j] = t & M;
        b = t >> 31;
        any |= d[j];
    }
    uint32_t k = grp_carry_in<G>(b != 0, any == 0u);
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const uint32_t t = d[j] - k;
        d[j] = t & M;
        k = t >> 31;
    }
    return grp_top_flag<G>((b | k) != 0) ? 1u : 0u;
}

template <int S, int G, int B>
__device__ __forceinline__ void rgrp_cond_sub(uint32_t (&x)[S / G], uint32_t top, const uint32_t (&n)[S / G])
{
    constexpr int L = S / G;
    uint32_t d[L];
    const uint32_t borrow = rgrp_sub<S, G, B>(d, x, n);
    const bool take = grp_top_flag<G>(top != 0) || !borrow;
#pragma unroll
    for (int j = 0; j < L; ++j) x[j] = take ? d[j] : x[j];
}

template <int S, int G, int B>
__device__ __forceinline__ void rgrp_dbl_mod(uint32_t (&x)[S / G], const uint32_t (&n)[S / G])
{
    constexpr int L = S / G;
    constexpr uint32_t M = Radix<B>::MASK;
    const uint32_t out = x[L - 1] >> (B - 1);
    const uint32_t in = grp_from_below<G>(out);
#pragma unroll
    for (int j = L - 1; j > 0; --j) x[j] = ((x[j] << 1) & M) | (x[j - 1] >> (B - 1));
    x[0] = ((x[0] << 1) & M) | in;
    rgrp_cond_sub<S, G, B>(x, out, n);
}

template <int S, int G, int B>
__device__ __forceinline__ uint32_t rgrp_bitlen(const uint32_t (&x)[S / G])
{
    constexpr int L = S / G;
    uint32_t bl = 0;
#pragma unroll
    for (int j = 0; j < L; ++j)
        if (x[j]) bl = (uint32_t)(B * (grp_lane<G>() * L + j) + 32 - __clz(x[j]));
    return grp_max<G>(bl);
}

// Sum over the group of one double per lane.  Every lane receives a sum of
// all G values, but the order, and so the rounding, may differ between lanes:
// a caller that needs one value takes lane 0's.
template <int G>
__device__ __forceinline__ double grp_sum_f64(double v)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, G);
    return v;
}

// (x + top * 2^(B*S)) / 2^e in double precision, for e near the value's bit
// length (the top word is the group's top lane's; limbs far below 2^e
// underflow harmlessly).
template <int S, int G, int B>
__device__ __forceinline__ double rgrp_scaled(const uint32_t (&x)[S / G], uint32_t top, int e)
{
    constexpr int L = S / G;
    const int r = grp_lane<G>();
    double part = r == G - 1 ? ldexp((double)top, B * S - e) : 0.0;
#pragma unroll
    for (int j = L - 1; j >= 0; --j) part += ldexp((double)x[j], B * (r * L + j) - e);
    return grp_sum_f64<G>(part);
}

// ---- accumulator normalisation -----------------------------------------

// Full: canonical B-bit limbs in w, returns the group's overflow beyond S
// limbs (meaningful in the top lane).
template <int S, int G, int B>
__device__ __forceinline__ uint32_t racc_normalise(uint32_t (&w)[S / G], const uint64_t (&acc)[S / G])
{
    constexpr int L = S / G;
    constexpr uint32_t M = Radix<B>::MASK;
    static_assert(L >= 2, "at least two limbs per lane");
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const uint64_t t = acc[j] + c;
        w[j] = (uint32_t)t & M;
        c = t >> B;
    }
    const bool top = grp_lane<G>() == G - 1;
    const uint32_t rlo = grp_from_below<G>((uint32_t)c), rhi = grp_from_below<G>((uint32_t)(c >> 32));
    const uint64_t own = top ? c : 0;
    uint64_t t = (uint64_t)w[0] + (((uint64_t)rhi << 32) | rlo);
    w[0] = (uint32_t)t & M;
    uint32_t k = (uint32_t)(t >> B);
#pragma unroll
    for (int j = 1; j < L; ++j) {
        const uint32_t u = w[j] + k;
        w[j] = u & M;
        k = u >> B;
    }
    bool all = true;
#pragma unroll
    for (int j = 0; j < L; ++j) all = all && w[j] == M;
    uint32_t k2 = grp_carry_in<G>(k != 0, all);
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const uint32_t u = w[j] + k2;
        w[j] = u & M;
        k2 = u >> B;
    }
    return top ? ((own != 0) | k | k2) : 0u;
}

// Redundant: limbs below 2^B + 2^(64-2B) holding the accumulator's value,
// for values below 2^(B*S) (nothing leaves the group's top lane).  Two rounds
// of "keep the low B bits, hand the rest to the next position": after the
// first every position is below 2^B + 2^(64-B), after the second below
// 2^B + 2^(64-2B).  Every position is independent within a round, so the
// dependency chain is a few instructions long instead of one carry chain
// through all S limbs; a Montgomery product accepts such limbs as inputs.
template <int S, int G, int B>
__device__ __forceinline__ void racc_lazy(uint32_t (&w)[S / G], const uint64_t (&acc)[S / G])
{
    constexpr int L = S / G;
    constexpr uint32_t M = Radix<B>::MASK;
    uint64_t v[L];
    {
        uint64_t hi[L];
#pragma unroll
        for (int j = 0; j < L; ++j) hi[j] = acc[j] >> B;
        const uint32_t in_lo = grp_from_below<G>((uint32_t)hi[L - 1]);
        const uint32_t in_hi = grp_from_below<G>((uint32_t)(hi[L - 1] >> 32));
        v[0] = (uint64_t)((uint32_t)acc[0] & M) + (((uint64_t)in_hi << 32) | in_lo);
#pragma unroll
        for (int j = 1; j < L; ++j) v[j] = (uint64_t)((uint32_t)acc[j] & M) + hi[j - 1];
    }
    uint32_t h2[L];
#pragma unroll
    for (int j = 0; j < L; ++j) h2[j] = (uint32_t)(v[j] >> B);
    const uint32_t in2 = grp_from_below<G>(h2[L - 1]);
    w[0] = ((uint32_t)v[0] & M) + in2;
#pragma unroll
    for (int j = 1; j < L; ++j) w[j] = ((uint32_t)v[j] & M) + h2[j - 1];
}

// x = x * 2^c mod n for canonical x < n, n < 2^(B*S - 10) and 1 <= c <= B - 1,
// given rn = 2^bl / n in double precision (bl the bit length of n).  y =
// x * 2^c is S limbs plus a top word (the bits beyond them, in the group's top
// lane).  q = floor(y / n) - 2 .. floor(y / n) comes from the doubles y / 2^bl
// and rn: their product is y / n within a relative 2^-45 and y / n < 2^c, so
// it is off by less than one, and q is its floor lowered by one (never below
// zero), taken from the group's lane 0 so that every lane subtracts the same
// q * n.  Then y - q * n < 3n fits S limbs, so it is the S-limb difference
// modulo 2^(B*S), and at most two subtractions of n make it canonical.  One
// call replaces c modular doublings (one carry chain each) by one multiply by
// a limb and three carry chains.
template <int S, int G, int B>
__device__ __forceinline__ void rgrp_shl_mod(uint32_t (&x)[S / G], uint32_t c, const uint32_t (&n)[S / G], double rn,
                                             int bl)
{
    constexpr int L = S / G;
    constexpr uint32_t M = Radix<B>::MASK;
    const uint32_t out = x[L - 1] >> (B - c);           // bits leaving this lane's top limb
    const uint32_t in = grp_from_below<G>(out);
    uint32_t y[L];
#pragma unroll
    for (int j = L - 1; j > 0; --j) y[j] = ((x[j] << c) & M) | (x[j - 1] >> (B - c));
    y[0] = ((x[0] << c) & M) | in;
    const uint32_t top = grp_lane<G>() == G - 1 ? out : 0u;
    double qd = floor(rgrp_scaled<S, G, B>(y, top, bl) * rn) - 1.0;
    qd = qd > 0.0 ? qd : 0.0;
    const uint32_t q = grp_bcast0<G>((uint32_t)qd);
    // q * n from 32-bit halves: a 64-bit product of the zero-extended limbs
    // here would let the compiler share the extension of n with the
    // exponentiation's products and lower those less well
    uint64_t acc[L];
#pragma unroll
    for (int j = 0; j < L; ++j) acc[j] = ((uint64_t)__umulhi(q, n[j]) << 32) | (uint32_t)(q * n[j]);
    uint32_t z[L];
    (void)racc_normalise<S, G, B>(z, acc);              // q * n modulo 2^(B*S)
    (void)rgrp_sub<S, G, B>(x, y, z);                   // y - q * n, exact below 2^(B*S)
    rgrp_cond_sub<S, G, B>(x, 0u, n);
    rgrp_cond_sub<S, G, B>(x, 0u, n);
}

// ---- Montgomery product, radix 2^B -----------------------------------------

// Reduction half of CIOS step k of a block: m from the group's lowest
// position (lane 0, register k), m * n into the rotating positions, the
// lowest register's carry into the next and its low B bits one lane down.
template <int S, int G, int B>
__device__ __forceinline__ void rcios_reduce(uint64_t (&acc)[S / G], int k, const uint32_t (&n)[S / G],
                                             uint32_t n0inv)
{
    constexpr int L = S / G;
    constexpr uint32_t M = Radix<B>::MASK;
    const int p0 = k % L, p1 = (k + 1) % L;
    // The masks follow the lane moves so that each pair folds into one
    // DPP-modified AND.
    const uint32_t Mv = vgpr_const(M);
    const uint32_t m = grp_bcast0_and<G>((uint32_t)acc[p0] * n0inv, Mv);
#pragma unroll
    for (int j = 0; j < L; ++j) acc[(j + k) % L] += (uint64_t)m * n[j];
    acc[p1] += acc[p0] >> B;
    // the group's lane 0 holds zero in its low B bits here
    acc[p0] = grp_rot_down_and<G>((uint32_t)acc[p0], Mv);
}

// The L CIOS steps of one block: multiplier limbs bv[0 .. L) (already
// broadcast to the group), accumulator positions rotating through acc.
template <int S, int G, int B>
__device__ __forceinline__ void rcios_block(uint64_t (&acc)[S / G], const uint32_t (&a)[S / G],
                                            const uint32_t (&bv)[S / G], const uint32_t (&n)[S / G],
                                            uint32_t n0inv)
{
    constexpr int L = S / G;
#pragma unroll
    for (int k = 0; k < L; ++k) {
#pragma unroll
        for (int j = 0; j < L; ++j) acc[(j + k) % L] += (uint64_t)a[j] * bv[k];
        rcios_reduce<S, G, B>(acc, k, n, n0inv);
    }
}

// Limbs per lane for which no accumulator can overflow: a register gathers
// at most 2L products below 2^(2B) * (1 + 2^-20) (inputs may carry redundant
// limbs) plus a carry below 2^(64-B) and a limb below 2^B+2^(64-2B) between
// two drains.
template <int B, int L>
constexpr bool rdrain_fits()
{
    return L >= 1 && L <= ((1 << (64 - 2 * B)) - 2) / 2;
}

template <int S, int G, int B, bool LAZY>
__device__ __forceinline__ void rmont_finish(uint32_t (&r)[S / G], const uint64_t (&acc)[S / G],
                                             const uint32_t (&n)[S / G])
{
    if constexpr (LAZY) {
        racc_lazy<S, G, B>(r, acc);
    } else {
        const uint32_t top = racc_normalise<S, G, B>(r, acc);
        rgrp_cond_sub<S, G, B>(r, top, n);
    }
}

// r = a * b * 2^(-B*S) mod n for a < 2^(BS) in registers and b < n in the
// group's slot of LDS buffer bbuf (or a < n, b < 2^(BS)); n0inv = -n^-1 mod 2^B.
//
// LAZY: no final subtraction and redundant output limbs (racc_lazy).  For
// a, b < 2n the result a*b/R + m*n/R is below 2n as long as R > 4n, which
// every width class gives with room to spare (R >= 2^10 * n), so a chain of
// lazy products stays below 2n without ever comparing with n; inputs may
// have redundant limbs (below 2^B + 2^(64-2B)): the products stay below
// 2^(2B) * (1 + 2^-20), which the accumulator bound (rdrain_fits) allows
// for.  The canonical form is restored by one non-lazy product (leaving the
// Montgomery domain does exactly that).
template <int S, int G, int B, bool LAZY = false>
__device__ __forceinline__ void rmont_mul(uint32_t (&r)[S / G], const uint32_t (&a)[S / G], const uint32_t *bbuf,
                                          const uint32_t (&n)[S / G], uint32_t n0inv)
{
    using Ly = Layout<S, G>;
    constexpr int L = Ly::L, V = Ly::V;
    static_assert(rdrain_fits<B, L>(), "limbs per lane too large for the radix");
    const int g = grp_index<G>();
    uint64_t acc[L];
#pragma unroll
    for (int j = 0; j < L; ++j) acc[j] = 0;

    for (int i0 = 0; i0 < S; i0 += L) {
        uint32_t bv[L];
#pragma unroll
        for (int k = 0; k < L; k += V) {
            typename VecT<V>::T v = *reinterpret_cast<const typename VecT<V>::T *>(bbuf + Ly::at(i0 + k, g));
            const uint32_t *pv = reinterpret_cast<const uint32_t *>(&v);
#pragma unroll
            for (int u = 0; u < V; ++u) bv[k + u] = pv[u];
        }
        rcios_block<S, G, B>(acc, a, bv, n, n0inv);
    }
    rmont_finish<S, G, B, LAZY>(r, acc, n);
}

// Blocks Q .. G-1 of a product whose multiplier b is held in the group's
// registers like a: block Q takes limbs Q*L .. Q*L+L-1, which lane Q holds.
template <int S, int G, int B, int Q>
struct RRegBlocks {
    static __device__ __forceinline__ void run(uint64_t (&acc)[S / G], const uint32_t (&a)[S / G],
                                               const uint32_t (&b)[S / G], const uint32_t (&n)[S / G],
                                               uint32_t n0inv)
    {
        if constexpr (Q < G) {
            constexpr int L = S / G;
            uint32_t bv[L];
#pragma unroll
            for (int k = 0; k < L; ++k) bv[k] = grp_bcast_lane<G, Q>(b[k]);
            rcios_block<S, G, B>(acc, a, bv, n, n0inv);
            RRegBlocks<S, G, B, Q + 1>::run(acc, a, b, n, n0inv);
        }
    }
};

// r = a * b * 2^(-B*S) mod n with both operands in the group's registers and
// the multiplier limbs broadcast by DPP (no LDS round trip); G = 2, 4 or 16.
// Same bounds and LAZY meaning as rmont_mul; r may alias a or b.
template <int S, int G, int B, bool LAZY>
__device__ __forceinline__ void rmont_mul_regs(uint32_t (&r)[S / G], const uint32_t (&a)[S / G],
                                               const uint32_t (&b)[S / G], const uint32_t (&n)[S / G],
                                               uint32_t n0inv)
{
    constexpr int L = S / G;
    static_assert(rdrain_fits<B, L>(), "limbs per lane too large for the radix");
    uint64_t acc[L];
#pragma unroll
    for (int j = 0; j < L; ++j) acc[j] = 0;
    RRegBlocks<S, G, B, 0>::run(acc, a, b, n, n0inv);
    rmont_finish<S, G, B, LAZY>(r, acc, n);
}

// Limbs per lane for which a squaring (rmont_sqr_regs) cannot overflow an
// accumulator: its products carry a factor 2, so a register gathers at most
// L products below 2^(2B+1) * (1 + 2^-20) and L below 2^(2B) * (1 + 2^-20)
// between two drains, plus the carry and the limb.
template <int B, int L>
constexpr bool rsqr_fits()
{
    return L >= 1 && 3 * L <= (1 << (64 - 2 * B)) - 2;
}

// Block Q of a Montgomery squaring: steps Q*L .. Q*L+L-1 take the group's
// own limbs of lane Q as multipliers.  A square needs each unordered pair of
// limbs once, doubled, and each limb squared once.  Lane r, register j, step
// k of block Q multiplies limbs Q*L+k and r*L+j; the pair with the other
// order of offsets (register k, step j of block r) is the same unordered
// pair, so only registers j >= k run: j > k with the doubled multiplier for
// every lane, and j == k per lane -- the square of the lane's own limb in
// lane Q, the doubled pair in lanes above Q, nothing in lanes below Q (they
// take that pair in their own block).  Every column still receives all its
// terms no later than its drain, so m and the result are those of the
// general product rcios_block computes with b = a; a2 holds 2a.
//
// The j == k multiplier is taken from the doubled limb b2 = 2 * limb < 2^31
// (limbs, redundant ones included, are below 2^30) by one bit-field
// extract whose per-lane offset and width are fixed for the block: b2 above
// lane Q (offset 0, width 31), b2 / 2 -- lane Q's own limb -- in lane Q
// (offset 1, width 31), 0 below (width 0).
__device__ __forceinline__ uint32_t diag_mult(uint32_t b2, uint32_t off, uint32_t wid)
{
    return __builtin_amdgcn_ubfe(b2, off, wid);
}

template <int S, int G, int B, int Q>
struct RSqrBlocks {
    static __device__ __forceinline__ void run(uint64_t (&acc)[S / G], const uint32_t (&a)[S / G],
                                               const uint32_t (&a2)[S / G], const uint32_t (&n)[S / G],
                                               uint32_t n0inv)
    {
        if constexpr (Q < G) {
            constexpr int L = S / G;
            const int r = grp_lane<G>();
            const uint32_t off = r == Q ? 1u : 0u, wid = r >= Q ? 31u : 0u;
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const uint32_t b2 = grp_bcast_lane<G, Q>(a2[k]);
                const uint32_t bd = diag_mult(b2, off, wid);
                acc[(2 * k) % L] += (uint64_t)a[k] * bd;
#pragma unroll
                for (int j = k + 1; j < L; ++j) acc[(j + k) % L] += (uint64_t)a[j] * b2;
                rcios_reduce<S, G, B>(acc, k, n, n0inv);
            }
            RSqrBlocks<S, G, B, Q + 1>::run(acc, a, a2, n, n0inv);
        }
    }
};

// r = a * a * 2^(-B*S) mod n with a in the group's registers (G = 2, 4 or 16):
// S * (L + 1) / 2 products per lane for the square instead of S * L.  Same
// bounds and LAZY meaning as rmont_mul; r may alias a.
template <int S, int G, int B, bool LAZY>
__device__ __forceinline__ void rmont_sqr_regs(uint32_t (&r)[S / G], const uint32_t (&a)[S / G],
                                               const uint32_t (&n)[S / G], uint32_t n0inv)
{
    constexpr int L = S / G;
    static_assert(rsqr_fits<B, L>(), "limbs per lane too large for a squaring in this radix");
    uint32_t a2[L];
#pragma unroll
    for (int k = 0; k < L; ++k) a2[k] = a[k] << 1;
    uint64_t acc[L];
#pragma unroll
    for (int j = 0; j < L; ++j) acc[j] = 0;
    RSqrBlocks<S, G, B, 0>::run(acc, a, a2, n, n0inv);
    rmont_finish<S, G, B, LAZY>(r, acc, n);
}

// The same squaring with the group's limbs of a also staged in its slot of
// LDS buffer abuf (any G): block q reads lane q's limbs there instead of
// broadcasting them by DPP.
template <int S, int G, int B, bool LAZY>
__device__ __forceinline__ void rmont_sqr(uint32_t (&r)[S / G], const uint32_t (&a)[S / G], const uint32_t *abuf,
                                          const uint32_t (&n)[S / G], uint32_t n0inv)
{
    using Ly = Layout<S, G>;
    constexpr int L = Ly::L, V = Ly::V;
    static_assert(rsqr_fits<B, L>(), "limbs per lane too large for a squaring in this radix");
    const int g = grp_index<G>(), lane = grp_lane<G>();
    uint64_t acc[L];
#pragma unroll
    for (int j = 0; j < L; ++j) acc[j] = 0;
    for (int q = 0; q < G; ++q) {
        uint32_t bv[L];
#pragma unroll
        for (int k = 0; k < L; k += V) {
            typename VecT<V>::T v = *reinterpret_cast<const typename VecT<V>::T *>(abuf + Ly::at(q * L + k, g));
            const uint32_t *pv = reinterpret_cast<const uint32_t *>(&v);
#pragma unroll
            for (int u = 0; u < V; ++u) bv[k + u] = pv[u];
        }
        const uint32_t off = lane == q ? 1u : 0u, wid = lane >= q ? 31u : 0u;
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const uint32_t b2 = bv[k] << 1;
            const uint32_t bd = diag_mult(b2, off, wid);
            acc[(2 * k) % L] += (uint64_t)a[k] * bd;
#pragma unroll
            for (int j = k + 1; j < L; ++j) acc[(j + k) % L] += (uint64_t)a[j] * b2;
            rcios_reduce<S, G, B>(acc, k, n, n0inv);
        }
    }
    rmont_finish<S, G, B, LAZY>(r, acc, n);
}

// (low, high) = init + a * b (no reduction), b in LDS; lane 0 of the group
// passes low limb i to sink(i, limb); high gets the upper S limbs.
template <int S, int G, int B, typename Sink>
__device__ __forceinline__ void rmul_wide(uint32_t (&high)[S / G], const uint32_t (&init)[S / G],
                                          const uint32_t (&a)[S / G], const uint32_t *bbuf, Sink sink)
{
    using Ly = Layout<S, G>;
    constexpr int L = Ly::L, V = Ly::V;
    constexpr uint32_t M = Radix<B>::MASK;
    static_assert(rdrain_fits<B, L>(), "limbs per lane too large for the radix");
    const int g = grp_index<G>();
    uint64_t acc[L];
#pragma unroll
    for (int j = 0; j < L; ++j) acc[j] = init[j];

    for (int i0 = 0; i0 < S; i0 += L) {
        uint32_t bv[L];
#pragma unroll
        for (int k = 0; k < L; k += V) {
            typename VecT<V>::T v = *reinterpret_cast<const typename VecT<V>::T *>(bbuf + Ly::at(i0 + k, g));
            const uint32_t *pv = reinterpret_cast<const uint32_t *>(&v);
#pragma unroll
            for (int u = 0; u < V; ++u) bv[k + u] = pv[u];
        }
#pragma unroll
        for (int k = 0; k < L; ++k) {
#pragma unroll
            for (int j = 0; j < L; ++j) acc[(j + k) % L] += (uint64_t)a[j] * bv[k];
            const int p0 = k % L, p1 = (k + 1) % L;
            sink(i0 + k, (uint32_t)acc[p0] & M);
            acc[p1] += acc[p0] >> B;
            acc[p0] = grp_from_above<G>((uint32_t)acc[p0] & M);
        }
    }
    racc_normalise<S, G, B>(high, acc);
}

}  // namespace rsagpu
