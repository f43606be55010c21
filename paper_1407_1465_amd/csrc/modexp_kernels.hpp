// Batched modular-exponentiation kernels for gfx950.
//
// A 64-lane workgroup (one wave) holds NG = 64 / G exponentiations, one per
// lane group.  The per-wave LDS holds the sliding window's table of odd
// powers T[k] = x^(2k+1) (paper, Section 3.6.5, a refinement of the k-ary
// method of Section 3.6.4) and, where the multiplier of a product is read
// from LDS, one operand buffer; each entry is one S-limb integer per group.
//
// The kernels are generic over the limb radix 2^B: B = 32 uses the carry-
// tracking arithmetic of group_bn.hpp, B < 32 the carry-free accumulation of
// radix_bn.hpp.  Inputs and outputs are always 32-bit-limb integers.
#pragma once

#include "group_bn.hpp"
#include "radix_bn.hpp"
#include "launch.hpp"

// Minimum waves per SIMD a plain exponentiation kernel is compiled for (the
// register budget per lane is 512 / waves).  With 14 or more limbs per lane
// the unconstrained allocation exceeds 256 registers, one wave per SIMD;
// capping it at two waves costs a few spills outside the product loop and
// hides the loop's dependency chains behind a second wave.  The CRT kernels
// are left unconstrained: at their best windows the LDS table already limits
// them to one wave per SIMD.
template <int L>
constexpr int exp_waves_per_simd() { return L >= 14 ? 2 : 1; }
#define RSAGPU_EXP_OCC(L) __attribute__((amdgpu_waves_per_eu(exp_waves_per_simd<(L)>())))

namespace rsagpu {

extern __shared__ uint4 rsagpu_lds[];

// Arithmetic of one lane group in radix 2^B.
template <int S, int G, int B>
struct Arith {
    static constexpr int L = S / G;
    static __device__ __forceinline__ uint32_t n0inv(uint32_t n0) { return neg_inv32(n0) & Radix<B>::MASK; }
    static __device__ __forceinline__ void load(uint32_t (&x)[L], const uint32_t *p, int nwords, int bitoff,
                                                bool live)
    {
        rload<S, G, B>(x, p, nwords, bitoff, live);
    }
    static __device__ __forceinline__ void mont_mul(uint32_t (&r)[L], const uint32_t (&a)[L], const uint32_t *b,
                                                    const uint32_t (&n)[L], uint32_t n0inv)
    {
        rmont_mul<S, G, B>(r, a, b, n, n0inv);
    }
    // Result below 2n with redundant limbs (see rmont_mul); inputs likewise.
    static __device__ __forceinline__ void mont_mul_lazy(uint32_t (&r)[L], const uint32_t (&a)[L],
                                                         const uint32_t *b, const uint32_t (&n)[L], uint32_t n0inv)
    {
        rmont_mul<S, G, B, true>(r, a, b, n, n0inv);
    }
    // Lazy product with the multiplier in the group's registers (G = 2, 4 or 16).
    static __device__ __forceinline__ void mont_mul_regs_lazy(uint32_t (&r)[L], const uint32_t (&a)[L],
                                                              const uint32_t (&b)[L], const uint32_t (&n)[L],
                                                              uint32_t n0inv)
    {
        rmont_mul_regs<S, G, B, true>(r, a, b, n, n0inv);
    }
    // The same product with a canonical result (below n, canonical limbs).
    static __device__ __forceinline__ void mont_mul_regs(uint32_t (&r)[L], const uint32_t (&a)[L],
                                                         const uint32_t (&b)[L], const uint32_t (&n)[L],
                                                         uint32_t n0inv)
    {
        rmont_mul_regs<S, G, B, false>(r, a, b, n, n0inv);
    }
    // Lazy squares, symmetric (one product per limb pair) where kSqr: with a
    // in registers (G = 2, 4 or 16) or also staged in the group's slot of abuf.
    static constexpr bool kSqr = rsqr_fits<B, L>();
    static __device__ __forceinline__ void sqr_regs_lazy(uint32_t (&r)[L], const uint32_t (&a)[L],
                                                         const uint32_t (&n)[L], uint32_t n0inv)
    {
        if constexpr (kSqr && (G == 2 || G == 4 || G == 16)) rmont_sqr_regs<S, G, B, true>(r, a, n, n0inv);
        else rmont_mul_regs<S, G, B, true>(r, a, a, n, n0inv);
    }
    static __device__ __forceinline__ void sqr_lds_lazy(uint32_t (&r)[L], const uint32_t (&a)[L],
                                                        const uint32_t *abuf, const uint32_t (&n)[L],
                                                        uint32_t n0inv)
    {
        if constexpr (kSqr) rmont_sqr<S, G, B, true>(r, a, abuf, n, n0inv);
        else rmont_mul<S, G, B, true>(r, a, abuf, n, n0inv);
    }
    template <typename Sink>
    static __device__ __forceinline__ void mul_wide(uint32_t (&hi)[L], const uint32_t (&init)[L],
                                                    const uint32_t (&a)[L], const uint32_t *b, Sink sink)
    {
        rmul_wide<S, G, B>(hi, init, a, b, sink);
    }
    static __device__ __forceinline__ uint32_t add(uint32_t (&x)[L], const uint32_t (&y)[L])
    {
        return rgrp_add<S, G, B>(x, y);
    }
    static __device__ __forceinline__ uint32_t sub(uint32_t (&d)[L], const uint32_t (&x)[L], const uint32_t (&y)[L])
    {
        return rgrp_sub<S, G, B>(d, x, y);
    }
    static __device__ __forceinline__ void cond_sub(uint32_t (&x)[L], uint32_t top, const uint32_t (&n)[L])
    {
        rgrp_cond_sub<S, G, B>(x, top, n);
    }
    static __device__ __forceinline__ void dbl_mod(uint32_t (&x)[L], const uint32_t (&n)[L])
    {
        rgrp_dbl_mod<S, G, B>(x, n);
    }
    static __device__ __forceinline__ uint32_t bitlen(const uint32_t (&x)[L]) { return rgrp_bitlen<S, G, B>(x); }
};

template <int S, int G>
struct Arith<S, G, 32> {
    static constexpr int L = S / G;
    static __device__ __forceinline__ uint32_t n0inv(uint32_t n0) { return neg_inv32(n0); }
    static __device__ __forceinline__ void load(uint32_t (&x)[L], const uint32_t *p, int nwords, int bitoff,
                                                bool live)
    {
        const int r = grp_lane<G>(), w0 = bitoff >> 5;
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int w = w0 + r * L + k;
            x[k] = (live && w < nwords) ? p[w] : 0u;
        }
    }
    static __device__ __forceinline__ void mont_mul(uint32_t (&r)[L], const uint32_t (&a)[L], const uint32_t *b,
                                                    const uint32_t (&n)[L], uint32_t n0inv)
    {
        rsagpu::mont_mul<S, G>(r, a, b, n, n0inv);
    }
    // Radix 2^32 limbs are exact fits (2n may not fit S limbs): canonical.
    static __device__ __forceinline__ void mont_mul_lazy(uint32_t (&r)[L], const uint32_t (&a)[L],
                                                         const uint32_t *b, const uint32_t (&n)[L], uint32_t n0inv)
    {
        rsagpu::mont_mul<S, G>(r, a, b, n, n0inv);
    }
    static __device__ __forceinline__ void mont_mul_regs_lazy(uint32_t (&r)[L], const uint32_t (&a)[L],
                                                              const uint32_t (&b)[L], const uint32_t (&n)[L],
                                                              uint32_t n0inv)
    {
        rsagpu::mont_mul_regs<S, G>(r, a, b, n, n0inv);
    }
    static __device__ __forceinline__ void mont_mul_regs(uint32_t (&r)[L], const uint32_t (&a)[L],
                                                         const uint32_t (&b)[L], const uint32_t (&n)[L],
                                                         uint32_t n0inv)
    {
        rsagpu::mont_mul_regs<S, G>(r, a, b, n, n0inv);
    }
    static constexpr bool kSqr = false;
    static __device__ __forceinline__ void sqr_regs_lazy(uint32_t (&r)[L], const uint32_t (&a)[L],
                                                         const uint32_t (&n)[L], uint32_t n0inv)
    {
        rsagpu::mont_mul_regs<S, G>(r, a, a, n, n0inv);
    }
    static __device__ __forceinline__ void sqr_lds_lazy(uint32_t (&r)[L], const uint32_t (&a)[L],
                                                        const uint32_t *abuf, const uint32_t (&n)[L],
                                                        uint32_t n0inv)
    {
        rsagpu::mont_mul<S, G>(r, a, abuf, n, n0inv);
    }
    template <typename Sink>
    static __device__ __forceinline__ void mul_wide(uint32_t (&hi)[L], const uint32_t (&init)[L],
                                                    const uint32_t (&a)[L], const uint32_t *b, Sink sink)
    {
        rsagpu::mul_wide<S, G>(hi, init, a, b, sink);
    }
    static __device__ __forceinline__ uint32_t add(uint32_t (&x)[L], const uint32_t (&y)[L])
    {
        return grp_add<S, G>(x, y);
    }
    static __device__ __forceinline__ uint32_t sub(uint32_t (&d)[L], const uint32_t (&x)[L], const uint32_t (&y)[L])
    {
        return grp_sub<S, G>(d, x, y);
    }
    static __device__ __forceinline__ void cond_sub(uint32_t (&x)[L], uint32_t top, const uint32_t (&n)[L])
    {
        grp_cond_sub<S, G>(x, top, n);
    }
    static __device__ __forceinline__ void dbl_mod(uint32_t (&x)[L], const uint32_t (&n)[L]) { grp_dbl_mod<S, G>(x, n); }
    static __device__ __forceinline__ uint32_t bitlen(const uint32_t (&x)[L]) { return grp_bitlen<S, G>(x); }
};

// Writes the group's S-limb integer x (radix 2^B) as `nwords` 32-bit words at
// p (only when live; zeros when !valid).  For B < 32 the limbs go through the
// group's slot of the LDS staging area `stage` (S words per group).
template <int S, int G, int B>
__device__ __forceinline__ void store_words(uint32_t *p, const uint32_t (&x)[S / G], int nwords, bool live,
                                            bool valid, uint32_t *stage)
{
    constexpr int L = S / G;
    const int r = grp_lane<G>(), g = grp_index<G>();
    if constexpr (B == 32) {
        if (!live) return;
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int w = r * L + k;
            if (w < nwords) p[w] = valid ? x[k] : 0u;
        }
    } else {
        uint32_t *q = stage + g * S;
        lds_sync();
#pragma unroll
        for (int k = 0; k < L; ++k) q[r * L + k] = x[k];
        lds_sync();
        if (live)
            for (int w = r; w < nwords; w += G) p[w] = valid ? rword<B>(q, S, w) : 0u;
    }
}

// r = a * c * R^-1 mod n with c (registers) staged through the operand buffer.
template <int S, int G, int B>
__device__ __forceinline__ void mont_mul_reg(uint32_t (&r)[S / G], const uint32_t (&a)[S / G],
                                             const uint32_t (&c)[S / G], uint32_t *abuf,
                                             const uint32_t (&n)[S / G], uint32_t n0inv)
{
    lds_sync();
    lds_put<S, G>(abuf, c);
    lds_sync();
    Arith<S, G, B>::mont_mul(r, a, abuf, n, n0inv);
}

// A = A^2 * R^-1 mod n through the operand buffer.
template <int S, int G, int B>
__device__ __forceinline__ void mont_sqr(uint32_t (&A)[S / G], uint32_t *abuf, const uint32_t (&n)[S / G],
                                         uint32_t n0inv)
{
    mont_mul_reg<S, G, B>(A, A, A, abuf, n, n0inv);
}

// Montgomery constants of an odd modulus n > 1 in radix 2^B, R = 2^(B*S):
//   one = R mod n:   2^(bitlen(n)-1) moved up B*S - bitlen(n) + 1 bits;
//   r2 = R^2 mod n:  X = R * 2^e mod n throughout, ending at e = B*S: one
//                    moved up e0 bits, e0 the top bits of B*S, then
//                    left-to-right over its remaining bits X <- X*X/R (e
//                    doubles) and one doubling where the bit is set (e + 1).
// In radix 2^32 the moves up are modular doublings (a carry chain per bit);
// in the reduced radix (n < 2^(B*S - 10)) they go up to B - 1 bits at a time
// by rgrp_shl_mod (one multiply by a limb and three carry chains), so e0
// takes the top eight bits of B*S (128 <= e0 < 256) and four squarings fewer
// remain than with the top five.  REG_LADDER (the plain exponentiation
// kernel only): where the multiplier can come from registers, the squarings
// of that ladder are register products, lazy and symmetric between two
// squarings (2048-bit e = 65537 encryptions ~2% faster; in the CRT kernel
// the same change cost the exponentiation more than the set-up saved).
template <int S, int G, int B, bool REG_LADDER = false>
__device__ __forceinline__ void mont_setup(uint32_t (&one)[S / G], uint32_t (&r2)[S / G],
                                           const uint32_t (&n)[S / G], uint32_t n0inv, bool valid,
                                           uint32_t *abuf)
{
    using A = Arith<S, G, B>;
    constexpr int L = S / G;
    const uint32_t bl = A::bitlen(n);
    const int r = grp_lane<G>();
#pragma unroll
    for (int k = 0; k < L; ++k) one[k] = 0;
    if (valid) {
        const int top = (int)bl - 1;
#pragma unroll
        for (int k = 0; k < L; ++k)
            if (r * L + k == top / B) one[k] = 1u << (top % B);
    }
    const uint32_t nup = valid ? (uint32_t)(B * S) - bl + 1 : 0u;      // bits to move one up
    constexpr int E = B * S;
    constexpr int TOP = 31 - __builtin_clz((unsigned)E);
    if constexpr (B < 32) {
        const double rn = 1.0 / rgrp_scaled<S, G, B>(n, 0u, (int)bl);
        uint32_t left = nup;
#pragma unroll
        for (int step = 0; step < 2; ++step) {
            const uint32_t c = left < B - 1 ? left : (uint32_t)(B - 1);
            uint32_t y[L];
#pragma unroll
            for (int k = 0; k < L; ++k) y[k] = one[k];
            rgrp_shl_mod<S, G, B>(y, c ? c : 1u, n, rn, (int)bl);
#pragma unroll
            for (int k = 0; k < L; ++k) one[k] = c ? y[k] : one[k];
            left -= c;
        }
        const uint32_t maxd = wave_max(left);
        for (uint32_t t = 0; t < maxd; ++t) {
            uint32_t y[L];
#pragma unroll
            for (int k = 0; k < L; ++k) y[k] = one[k];
            A::dbl_mod(y, n);
            const bool act = t < left;
#pragma unroll
            for (int k = 0; k < L; ++k) one[k] = act ? y[k] : one[k];
        }
        constexpr int SH = TOP > 7 ? TOP - 7 : 0;      // E >> SH in [128, 256)
#pragma unroll
        for (int k = 0; k < L; ++k) r2[k] = one[k];
        for (int t = E >> SH; t > 0; t -= B - 1) rgrp_shl_mod<S, G, B>(r2, t < B - 1 ? t : B - 1, n, rn, (int)bl);
        if constexpr (REG_LADDER && register_products(B, G)) {
            // a squaring followed by another squaring is lazy and symmetric
            // (below 2n, redundant limbs); one followed by a doubling, or the
            // last, is canonical (a product of two values below 2n leaves
            // below 2n before its final subtraction, as R > 4n)
#pragma unroll
            for (int bit = SH - 1; bit >= 0; --bit) {
                const bool dbl = ((E >> bit) & 1) != 0;
                if (dbl || bit == 0) A::mont_mul_regs(r2, r2, r2, n, n0inv);
                else A::sqr_regs_lazy(r2, r2, n, n0inv);
                if (dbl) A::dbl_mod(r2, n);
            }
        } else {
            for (int bit = SH - 1; bit >= 0; --bit) {
                mont_sqr<S, G, B>(r2, abuf, n, n0inv);
                if ((E >> bit) & 1) A::dbl_mod(r2, n);
            }
        }
    } else {
        const uint32_t maxd = wave_max(nup);
        for (uint32_t t = 0; t < maxd; ++t) {
            uint32_t y[L];
#pragma unroll
            for (int k = 0; k < L; ++k) y[k] = one[k];
            A::dbl_mod(y, n);
            const bool act = t < nup;
#pragma unroll
            for (int k = 0; k < L; ++k) one[k] = act ? y[k] : one[k];
        }
        constexpr int SH = TOP > 4 ? TOP - 4 : 0;      // E >> SH in [16, 32)
#pragma unroll
        for (int k = 0; k < L; ++k) r2[k] = one[k];
        for (int t = 0; t < (E >> SH); ++t) A::dbl_mod(r2, n);
        for (int bit = SH - 1; bit >= 0; --bit) {
            mont_sqr<S, G, B>(r2, abuf, n, n0inv);
            if ((E >> bit) & 1) A::dbl_mod(r2, n);
        }
    }
}


// Exponent bits of one group, scanned from the top: `hi:lo` holds words kw
// and kw - 1 (bit positions 32*(kw-1) .. 32*kw+31) and `pre` word kw - 2,
// loaded a word ahead of its use.
struct ExpBits {
    const uint32_t *ep;
    int elimbs;
    int kw;
    uint64_t bits;
    uint32_t pre;

    __device__ __forceinline__ uint32_t word(int k) const { return (k >= 0 && k < elimbs) ? ep[k] : 0u; }
    __device__ __forceinline__ void start(int top)
    {
        kw = top >> 5;
        bits = ((uint64_t)word(kw) << 32) | word(kw - 1);
        pre = word(kw - 2);
    }
    // Makes bit `pos` (<= the previous pos) fall in the high word.
    __device__ __forceinline__ void seek(int pos)
    {
        if (pos >= 0 && (pos >> 5) < kw) {
            bits = (bits << 32) | pre;
            --kw;
            pre = word(kw - 2);
        }
    }
    // Bits lo .. hi (hi - lo < 32, hi in the high word, lo >= 32*(kw-1)).
    __device__ __forceinline__ uint32_t field(int hi, int lo) const
    {
        const int off = lo - 32 * (kw - 1);
        const uint32_t len = (uint32_t)(hi - lo + 1);
        return (uint32_t)(bits >> off) & (uint32_t)((1ull << len) - 1ull);
    }
};

// A = x^e mod n in Montgomery form, for xt = x*R mod n and an exponent e of
// elimbs 32-bit words at ep (read only when use_exp), by the left-to-right
// sliding window of Section 3.6.5 with windows of up to w bits: table of odd
// powers T[k] = x^(2k+1), k < 2^(w-1), in LDS (for exponents of at most 64
// bits only the powers the wave uses: 65537 needs x alone, 16 squarings and
// one product, as Fig. 5's binary method); a zero bit costs one squaring, a
// window of value v (odd) and length l costs l squarings and one product
// with T[(v-1)/2]; the leading window initialises A.  Each group runs its own
// schedule; the wave executes one Montgomery product per slot for all its
// groups, a squaring or a table product per group (the multiplier is
// selected per group), until every group is done, so the loop holds a single
// copy of the product.  With register_products(B, G) the multiplier comes
// from registers (DPP broadcast; the table starts at the LDS base); otherwise
// A is staged through the operand buffer at the LDS base (the table follows
// it) and each group's product reads its own multiplier there or in its
// table entry.  Where squarings can be symmetric (Arith::kSqr) and every
// live group of the wave has the same exponent words (one key's exponent,
// or a public exponent), the wave instead follows one schedule: its
// squarings multiply each pair of limbs once (rmont_sqr_regs, or rmont_sqr
// with A staged in the operand buffer) and its table products read one entry
// for all groups.  Every product is lazy (A and the
// table stay below 2n in redundant limbs); the caller's from_mont makes the
// result canonical.  With FUSE, x holds the base itself (not in Montgomery
// form): where the wave's one schedule ends with a product by T[0] = x R
// (an exponent whose last window is its lowest bit alone, such as 65537),
// that last product takes x instead and is not lazy, A * x / R = x^e mod n,
// canonical; group_modexp then returns true and the caller's from_mont is
// left out (one Montgomery product less).  It returns false otherwise.
template <int S, int G, int B, bool FUSE = false>
__device__ __forceinline__ bool group_modexp(uint32_t (&A)[S / G], const uint32_t (&xt)[S / G],
                                                     const uint32_t *ep, int elimbs, bool use_exp,
                                                     const uint32_t (&n)[S / G], uint32_t n0inv,
                                                     const uint32_t (&one)[S / G], uint32_t *lds, int w,
                                                     const uint32_t (&x)[S / G])
{
    using Ly = Layout<S, G>;
    using Ar = Arith<S, G, B>;
    constexpr int L = Ly::L;
    constexpr bool REG = register_products(B, G);
    uint32_t *abuf = lds;                       // operand buffer (LDS-multiplier products)
    uint32_t *tbl = REG ? lds : lds + Ly::WORDS;   // entry k at tbl + k * WORDS
    const int g = grp_index<G>();
    // lazy product with a multiplier in registers (b) or in LDS (bl)
    auto mul_regs = [&](uint32_t (&r)[L], const uint32_t (&a)[L], const uint32_t (&b)[L]) {
        if constexpr (REG) Ar::mont_mul_regs_lazy(r, a, b, n, n0inv);
    };
    auto mul_lds = [&](uint32_t (&r)[L], const uint32_t (&a)[L], const uint32_t *bl) {
        Ar::mont_mul_lazy(r, a, bl, n, n0inv);
    };

    // this group's exponent length (its lanes scan slices of the words) and,
    // where squarings can be symmetric, whether every live group of the wave
    // has group 0's exponent: then the whole wave follows one schedule
    constexpr bool UNI = Ar::kSqr;
    const int el = use_exp ? elimbs : 0;
    uint32_t ebits = 0;
    bool same = true;
    {
        const int per = ((int)wave_max((uint32_t)el) + G - 1) / G;
        const int r = grp_lane<G>();
        for (int k = 0; k < per; ++k) {
            const int li = r * per + k;
            const uint32_t v = li < el ? ep[li] : 0u;
            if (v) ebits = (uint32_t)(32 * li + 32 - __clz(v));
            if constexpr (UNI) same = same && (!use_exp || v == (uint32_t)__shfl((int)v, r));
        }
    }
    ebits = grp_max<G>(ebits);
    const bool uniform = UNI && __ballot(!same) == 0;

    ExpBits eb{ep, use_exp ? elimbs : 0, 0, 0, 0};
    int pos = (int)ebits - 1;                   // next bit to scan
    int sq = 0, mi = -1;                        // pending squarings, pending table index
    // Takes the next window at pos: a zero bit (one squaring) or a window
    // ending in a one (its length in squarings, then T[(v-1)/2]).  (Taking
    // whole runs of zero bits at once measured slower: the extra scanning
    // code costs more than the calls it saves.)
    auto next_window = [&]() {
        eb.seek(pos);
        if (((uint32_t)(eb.bits >> (pos - 32 * (eb.kw - 1))) & 1u) == 0u) {
            sq = 1;
            mi = -1;
            pos -= 1;
            return;
        }
        const int lo0 = pos - w + 1 > 0 ? pos - w + 1 : 0;
        uint32_t v = eb.field(pos, lo0);
        const int tz = __builtin_ctz(v);
        v >>= tz;
        sq = pos - (lo0 + tz) + 1;
        mi = (int)(v >> 1);
        pos = lo0 + tz - 1;
    };

    // Table size: all 2^(w-1) odd powers, or for short exponents (public
    // exponents such as 65537) only those the wave's schedules use, found by
    // one scan of the windows without products.
    int tsize = 1 << (w - 1);
    if (wave_max(ebits) <= 64u) {
        int used = 0;
        if (pos >= 0) {
            eb.start(pos);
            while (pos >= 0) {
                next_window();
                used = mi + 1 > used ? mi + 1 : used;
            }
        }
        tsize = (int)wave_max((uint32_t)used);
        pos = (int)ebits - 1;
        sq = 0;
        mi = -1;
    }

    // odd powers: T[0] = x, T[k] = T[k-1] * x^2
    {
        uint32_t cur[L];
#pragma unroll
        for (int k = 0; k < L; ++k) cur[k] = xt[k];
        lds_sync();                             // earlier users of the operand buffer are done
        lds_put<S, G>(tbl, cur);
        if (tsize > 1) {
            uint32_t x2[L];
            if constexpr (REG) {
                mul_regs(x2, xt, xt);
            } else {
                lds_sync();
                mul_lds(x2, xt, tbl);
                lds_put<S, G>(abuf, x2);
                lds_sync();
            }
            for (int i = 1; i < tsize; ++i) {
                if constexpr (REG) mul_regs(cur, cur, x2);
                else mul_lds(cur, cur, abuf);
                lds_put<S, G>(tbl + i * Ly::WORDS, cur);
            }
        }
        lds_sync();
    }

    if constexpr (UNI) {
        if (uniform) {
            // One schedule for the wave, group 0's (all live groups share its
            // exponent; the others' results are not used): squarings are
            // symmetric and no multiplier is selected per group.
            eb = ExpBits{first_lane_ptr(ep), __builtin_amdgcn_readfirstlane(el), 0, 0, 0};
            pos = __builtin_amdgcn_readfirstlane((int)ebits) - 1;
#pragma unroll
            for (int k = 0; k < L; ++k) A[k] = one[k];
            if (pos < 0) return false;
            eb.start(pos);
            next_window();                      // the leading window sets A
            lds_get<S, G>(A, tbl + __builtin_amdgcn_readfirstlane(mi) * Ly::WORDS, g);
            while (__builtin_amdgcn_readfirstlane(pos) >= 0) {
                next_window();
                const int nsq = __builtin_amdgcn_readfirstlane(sq), ui = __builtin_amdgcn_readfirstlane(mi);
                for (int q = 0; q < nsq; ++q) {
                    if constexpr (REG) {
                        Ar::sqr_regs_lazy(A, A, n, n0inv);
                    } else {
                        lds_sync();
                        lds_put<S, G>(abuf, A);
                        lds_sync();
                        Ar::sqr_lds_lazy(A, A, abuf, n, n0inv);
                    }
                }
                if constexpr (FUSE) {
                    if (ui == 0 && __builtin_amdgcn_readfirstlane(pos) < 0) {
                        if constexpr (REG) Ar::mont_mul_regs(A, A, x, n, n0inv);
                        else mont_mul_reg<S, G, B>(A, A, x, abuf, n, n0inv);
                        return true;
                    }
                }
                if (ui >= 0) {
                    if constexpr (REG) {
                        uint32_t tb[L];
                        lds_get<S, G>(tb, tbl + ui * Ly::WORDS, g);
                        mul_regs(A, A, tb);
                    } else {
                        mul_lds(A, A, tbl + ui * Ly::WORDS);
                    }
                }
            }
            return false;
        }
    }

#pragma unroll
    for (int k = 0; k < L; ++k) A[k] = one[k];
    if (pos >= 0) {
        eb.start(pos);
        next_window();                          // the leading bit is one: a window
        uint32_t t[L];
        lds_get<S, G>(t, tbl + mi * Ly::WORDS, g);
#pragma unroll
        for (int k = 0; k < L; ++k) A[k] = t[k];
        sq = 0;
        mi = -1;
        if (pos >= 0) next_window();
    }
    for (;;) {
        const bool active = sq > 0 || mi >= 0;
        if (!__ballot(active)) break;
        const bool mul = sq == 0 && mi >= 0;
        uint32_t t[L];
        if constexpr (REG) {
            uint32_t b[L];
#pragma unroll
            for (int k = 0; k < L; ++k) b[k] = A[k];
            if (__ballot(mul)) {
                uint32_t tb[L];                 // this lane's limbs of T[mi]
                lds_get<S, G>(tb, tbl + (mul ? mi : 0) * Ly::WORDS, g);
#pragma unroll
                for (int k = 0; k < L; ++k) b[k] = mul ? tb[k] : b[k];
            }
            mul_regs(t, A, b);
        } else {
            lds_sync();
            lds_put<S, G>(abuf, A);
            lds_sync();
            mul_lds(t, A, mul ? tbl + mi * Ly::WORDS : abuf);
        }
#pragma unroll
        for (int k = 0; k < L; ++k) A[k] = active ? t[k] : A[k];
        if (mul) mi = -1;
        else if (sq > 0) --sq;
        if (sq == 0 && mi < 0 && pos >= 0) next_window();
    }
    return false;
}

// A = A * R^-1 mod n (leave Montgomery form).
template <int S, int G, int B>
__device__ __forceinline__ void from_mont(uint32_t (&A)[S / G], uint32_t *abuf, const uint32_t (&n)[S / G],
                                          uint32_t n0inv)
{
    constexpr int L = S / G;
    uint32_t u[L];
#pragma unroll
    for (int k = 0; k < L; ++k) u[k] = (grp_lane<G>() == 0 && k == 0) ? 1u : 0u;
    mont_mul_reg<S, G, B>(A, A, u, abuf, n, n0inv);
}

// ---- out[i] = base[i]^exp[i] mod mod[i] --------------------------------
//
// S limbs of radix 2^B hold the caller's `limbs` 32-bit words (B*S >= 32*limbs).
template <int S, int G, int B>
__global__ __launch_bounds__(64) RSAGPU_EXP_OCC(S / G) void k_modexp(const uint32_t *__restrict__ base,
                                               const uint32_t *__restrict__ exp,
                                               const uint32_t *__restrict__ mod,
                                               uint32_t *out, unsigned long long count, int limbs, int w,
                                               unsigned long long *errs)
{
    using Ar = Arith<S, G, B>;
    constexpr int L = S / G, NG = 64 / G;
    uint32_t *lds = reinterpret_cast<uint32_t *>(rsagpu_lds);
    const int g = grp_index<G>(), r = grp_lane<G>();
    const unsigned long long msg = (unsigned long long)blockIdx.x * NG + g;
    const bool live = msg < count;
    const size_t off = live ? (size_t)msg * (size_t)limbs : 0;

    uint32_t n[L], x[L];
    Ar::load(n, mod + off, limbs, 0, live);
    Ar::load(x, base + off, limbs, 0, live);
    const uint32_t n0 = grp_bcast0<G>(n[0]);
    const uint32_t bl = Ar::bitlen(n);
    const bool valid = live && (n0 & 1u) && bl > 1;
    const uint32_t n0inv = Ar::n0inv(n0 | 1u);

    uint32_t one[L], r2[L], xt[L], A[L];
    mont_setup<S, G, B, true>(one, r2, n, n0inv, valid, lds);
    mont_mul_reg<S, G, B>(xt, x, r2, lds, n, n0inv);
    if (!group_modexp<S, G, B, true>(A, xt, exp + off, limbs, valid, n, n0inv, one, lds, w, x))
        from_mont<S, G, B>(A, lds, n, n0inv);

    store_words<S, G, B>(out + off, A, limbs, live, valid, lds);
    if (live && r == 0 && !valid && bl != 1) atomicAdd(errs, 1ull);
}

// ---- CRT decryption ------------------------------------------------------
//
// A pair of waves takes NG = 64 / G messages: the pair's wave 0 the halves
// modulo p, its wave 1 the halves modulo q, one message per lane group, so a
// wave's exponents are all dp (or all dq) and, when its messages share a key,
// equal (group_modexp then runs one schedule with symmetric squarings).  A
// workgroup holds P = blockDim.x / 128 pairs (1 or 2), which take consecutive
// runs of NG slots: slot i of pair j is (blockIdx.x * P + j) * NG + i, and
// holds message order[slot] (the identity without an order) unless that is
// kOrderHole; groups of empty slots compute nothing that is stored, and a
// workgroup of empty slots only returns at once.  p, q, dp, dq, qinv have hl
// 32-bit words, c
// and the result 2*hl; H limbs of radix 2^B hold a half (B*H >= 32*hl).
// Each wave works in its own LDS region; m_q and its validity reach the
// pair's wave 0 through its wave 1's region, and wave 0 recombines (Garner)
// and stores.
template <int H, int G, int B>
__global__ __launch_bounds__(256) void k_crt(
    const uint32_t *__restrict__ c, const uint32_t *__restrict__ p, const uint32_t *__restrict__ q,
    const uint32_t *__restrict__ dp, const uint32_t *__restrict__ dq, const uint32_t *__restrict__ qinv,
    const unsigned *__restrict__ order, uint32_t *out, unsigned long long count, int hl, int w,
    unsigned long long *errs)
{
    using Ar = Arith<H, G, B>;
    using Ly = Layout<H, G>;
    constexpr int L = H / G, NG = 64 / G;
    const int P = (int)(blockDim.x >> 7);
    const int wave = (int)(threadIdx.x >> 6), pair = wave >> 1, half = wave & 1;
    const size_t region = (size_t)lds_entries(B, G, w) * Ly::WORDS;
    uint32_t *lds = reinterpret_cast<uint32_t *>(rsagpu_lds) + wave * region;
    uint32_t *qlds = reinterpret_cast<uint32_t *>(rsagpu_lds) + (2 * pair + 1) * region;   // the pair's wave 1
    const int g = grp_index<G>(), r = grp_lane<G>();
    const unsigned long long slot = ((unsigned long long)blockIdx.x * P + pair) * NG + g;
    bool live = slot < count;
    unsigned long long msg = slot;
    if (live && order) {
        const unsigned o = order[slot];
        live = o != kOrderHole;
        msg = o;
    }
    if (!live) msg = 0ull;
    {   // a workgroup of empty slots only returns at once (every wave finds so alike)
        const unsigned long long first = (unsigned long long)blockIdx.x * P * NG;
        bool any = false;
        for (int k = (int)__lane_id(); k < P * NG; k += 64) {
            const unsigned long long s = first + (unsigned)k;
            any = any || (s < count && (!order || order[s] != kOrderHole));
        }
        if (__ballot(any) == 0) return;
    }
    const size_t hoff = live ? (size_t)msg * (size_t)hl : 0;
    const size_t foff = 2 * hoff;
    const int full = 2 * hl;

    uint32_t n[L], clo[L], chi[L];
    Ar::load(n, (half ? q : p) + hoff, hl, 0, live);
    Ar::load(clo, c + foff, full, 0, live);                   // c mod R
    Ar::load(chi, c + foff, full, B * H, live);               // c div R
    const uint32_t n0 = grp_bcast0<G>(n[0]);
    const uint32_t bl = Ar::bitlen(n);
    bool valid = live && (n0 & 1u) && bl > 1;
    if (!half) {   // p > q
        uint32_t other[L], d[L];
        Ar::load(other, q + hoff, hl, 0, live);
        const uint32_t lt = Ar::sub(d, n, other);
        bool nz = false;
#pragma unroll
        for (int k = 0; k < L; ++k) nz = nz || d[k] != 0u;
        valid = valid && !lt && grp_any<G>(nz);
    }
    const uint32_t n0inv = Ar::n0inv(n0 | 1u);

    uint32_t one[L], r2[L], r3[L];
    mont_setup<H, G, B>(one, r2, n, n0inv, valid, lds);
    mont_mul_reg<H, G, B>(r3, r2, r2, lds, n, n0inv);        // R^3 mod n

    // xt = c * R mod n = c_lo * R + c_hi * R * R  (c = c_lo + c_hi * R)
    uint32_t xt[L], t2[L];
    mont_mul_reg<H, G, B>(xt, clo, r2, lds, n, n0inv);
    mont_mul_reg<H, G, B>(t2, chi, r3, lds, n, n0inv);
    {
        const uint32_t ovf = Ar::add(xt, t2);
        Ar::cond_sub(xt, ovf, n);
    }

    uint32_t A[L];
    group_modexp<H, G, B>(A, xt, (half ? dq : dp) + hoff, hl, valid, n, n0inv, one, lds, w, xt);
    from_mont<H, G, B>(A, lds, n, n0inv);

    // wave 1 hands m_q and its validity to wave 0
    if (half) {
        lds_sync();
        lds_put<H, G>(qlds, A);
        if (r == 0) qlds[Ly::WORDS + g] = valid ? 1u : 0u;
    }
    __syncthreads();
    if (half) return;

    // Garner: h = qinv * (m_p - m_q) mod p, m = m_q + h * q
    uint32_t mq[L], qv[L], hh[L];
    lds_get<H, G>(mq, qlds, g);
    valid = valid && qlds[Ly::WORDS + g] != 0u;
    {   // delta = m_p - m_q mod p  (m_q < q < p)
        uint32_t d[L];
        const uint32_t neg = Ar::sub(d, A, mq);
        uint32_t e[L];
#pragma unroll
        for (int k = 0; k < L; ++k) e[k] = d[k];
        Ar::add(e, n);
#pragma unroll
        for (int k = 0; k < L; ++k) A[k] = neg ? e[k] : d[k];
    }
    Ar::load(qv, qinv + hoff, hl, 0, live);
    mont_mul_reg<H, G, B>(qv, qv, r2, lds, n, n0inv);         // qinv * R mod p
    mont_mul_reg<H, G, B>(hh, A, qv, lds, n, n0inv);          // delta * qinv mod p
    lds_sync();
    lds_put<H, G>(lds, hh);
    lds_sync();
    // m = m_q + h * q: 2H limbs, staged in LDS after the operand buffer
    uint32_t *stage = lds + Ly::WORDS + g * (2 * H);
    auto sink = [&](int i, uint32_t v) {
        if (r == 0) stage[i] = v;
    };
    uint32_t high[L], qn[L];
    Ar::load(qn, q + hoff, hl, 0, live);
    Ar::mul_wide(high, mq, qn, lds, sink);
#pragma unroll
    for (int k = 0; k < L; ++k) stage[H + r * L + k] = high[k];
    lds_sync();
    if (live) {
        uint32_t *o = out + foff;
        if constexpr (B == 32) {
            for (int wd = r; wd < full; wd += G) o[wd] = valid ? stage[wd] : 0u;
        } else {
            for (int wd = r; wd < full; wd += G) o[wd] = valid ? rword<B>(stage, 2 * H, wd) : 0u;
        }
    }
    if (live && r == 0 && !valid) atomicAdd(errs, 1ull);
}

}  // namespace rsagpu
