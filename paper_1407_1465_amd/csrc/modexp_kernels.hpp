// Batched modular-exponentiation kernels for gfx950.
//
// A 64-lane workgroup (one wave) holds NG = 64 / G exponentiations, one per
// lane group.  The per-wave LDS holds one operand buffer (the multiplier of
// the next Montgomery product) and the fixed-window table T[1 .. 2^w - 1],
// each entry one S-limb integer per group (paper, Section 3.6.4: left-to-right
// k-ary exponentiation with a precomputed table of the powers g^1 .. g^(2^k-1)).
#pragma once

#include "group_bn.hpp"

namespace rsagpu {

extern __shared__ uint4 rsagpu_lds[];

template <int N>
struct OddPart { static constexpr int value = (N % 2 == 0) ? OddPart<N / 2>::value : N; };
template <>
struct OddPart<0> { static constexpr int value = 1; };

template <int N>
struct Log2 { static constexpr int value = 1 + Log2<N / 2>::value; };
template <>
struct Log2<1> { static constexpr int value = 0; };

// Loads limbs [r*L, r*L + L) of a `limbs`-limb integer at p (zero beyond
// `limbs`, zero when !live).
template <int S, int G>
__device__ __forceinline__ void load_limbs(uint32_t (&x)[S / G], const uint32_t *p, int limbs, bool live)
{
    constexpr int L = S / G;
    const int r = grp_lane<G>();
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const int li = r * L + k;
        x[k] = (live && li < limbs) ? p[li] : 0u;
    }
}

template <int S, int G>
__device__ __forceinline__ void store_limbs(uint32_t *p, const uint32_t (&x)[S / G], int limbs, bool live,
                                            bool valid)
{
    constexpr int L = S / G;
    const int r = grp_lane<G>();
    if (!live) return;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const int li = r * L + k;
        if (li < limbs) p[li] = valid ? x[k] : 0u;
    }
}

// One Montgomery squaring of A through the operand buffer.
template <int S, int G>
__device__ __forceinline__ void mont_sqr_lds(uint32_t (&A)[S / G], uint32_t *abuf, const uint32_t (&n)[S / G],
                                             uint32_t n0inv)
{
    lds_sync();
    lds_put<S, G>(abuf, A);
    lds_sync();
    mont_mul<S, G>(A, A, abuf, n, n0inv);
}

// r = a * c * R^-1 mod n with c (registers) staged through the operand buffer.
template <int S, int G>
__device__ __forceinline__ void mont_mul_reg(uint32_t (&r)[S / G], const uint32_t (&a)[S / G],
                                             const uint32_t (&c)[S / G], uint32_t *abuf,
                                             const uint32_t (&n)[S / G], uint32_t n0inv)
{
    lds_sync();
    lds_put<S, G>(abuf, c);
    lds_sync();
    mont_mul<S, G>(r, a, abuf, n, n0inv);
}

// Montgomery constants of an odd modulus n > 1, R = 2^(32S):
//   one = R mod n          (2^(bitlen(n)-1) doubled 32S - bitlen(n) + 1 times)
//   r2  = R^2 mod n        (one doubled c times, then squared j times in
//                           Montgomery form, where c * 2^j = 32S)
template <int S, int G>
__device__ __forceinline__ void mont_setup(uint32_t (&one)[S / G], uint32_t (&r2)[S / G],
                                           const uint32_t (&n)[S / G], uint32_t n0inv, bool valid,
                                           uint32_t *abuf)
{
    constexpr int L = S / G;
    const uint32_t bl = grp_bitlen<S, G>(n);
    const int r = grp_lane<G>();
#pragma unroll
    for (int k = 0; k < L; ++k) one[k] = 0;
    if (valid) {
        const int top = (int)bl - 1;
#pragma unroll
        for (int k = 0; k < L; ++k)
            if (r * L + k == top / 32) one[k] = 1u << (top % 32);
    }
    const uint32_t ndbl = valid ? (uint32_t)(32 * S) - bl + 1 : 0u;
    const uint32_t maxd = wave_max(ndbl);
    for (uint32_t t = 0; t < maxd; ++t) {
        uint32_t y[L];
#pragma unroll
        for (int k = 0; k < L; ++k) y[k] = one[k];
        grp_dbl_mod<S, G>(y, n);
        const bool act = t < ndbl;
#pragma unroll
        for (int k = 0; k < L; ++k) one[k] = act ? y[k] : one[k];
    }
    constexpr int C = OddPart<S>::value;
    constexpr int J = Log2<(32 * S) / C>::value;
    static_assert(C * (1 << J) == 32 * S, "c * 2^j must be 32S");
#pragma unroll
    for (int k = 0; k < L; ++k) r2[k] = one[k];
    for (int t = 0; t < C; ++t) grp_dbl_mod<S, G>(r2, n);
    for (int t = 0; t < J; ++t) mont_sqr_lds<S, G>(r2, abuf, n, n0inv);
}

// Fixed-window digit of an exponent: bits [pos, pos + w) (zero beyond elimbs).
__device__ __forceinline__ uint32_t exp_digit(const uint32_t *ep, int elimbs, int pos, int w)
{
    const int li = pos >> 5, sh = pos & 31;
    const uint32_t lo = li < elimbs ? ep[li] : 0u;
    const uint32_t hi = (sh + w > 32 && li + 1 < elimbs) ? ep[li + 1] : 0u;
    const uint64_t v = (((uint64_t)hi << 32) | lo) >> sh;
    return (uint32_t)v & ((1u << w) - 1u);
}

// A = x^e mod n, returned in Montgomery form, for xt = x*R mod n in Montgomery
// form and exponent e of elimbs limbs at ep (read only when use_exp).
//
// Left-to-right k-ary method (Section 3.6.4, Fig. 6) with k = w: table
// T[i] = x^i (i = 1 .. 2^w - 1) in LDS, then, from the most significant
// digit, w squarings followed by one product with T[digit].  The leading
// digit initialises A directly (the w squarings of 1 are skipped); a zero
// digit skips its product.  The window count is the wave's largest exponent
// length, so groups with shorter exponents run on A = 1 until their digits
// start.
template <int S, int G>
__device__ __forceinline__ void group_modexp(uint32_t (&A)[S / G], const uint32_t (&xt)[S / G],
                                             const uint32_t *ep, int elimbs, bool use_exp,
                                             const uint32_t (&n)[S / G], uint32_t n0inv,
                                             const uint32_t (&one)[S / G], uint32_t *lds, int w)
{
    using Ly = Layout<S, G>;
    constexpr int L = Ly::L;
    uint32_t *abuf = lds;
    uint32_t *tbl = lds + Ly::WORDS;            // entry i at tbl + (i - 1) * WORDS
    const int g = grp_index<G>();
    const int r = grp_lane<G>();

    // table T[1] = x, T[i] = T[i-1] * x
    lds_sync();
    lds_put<S, G>(tbl, xt);
    uint32_t cur[L];
#pragma unroll
    for (int k = 0; k < L; ++k) cur[k] = xt[k];
    lds_sync();
    const int tsize = 1 << w;
    for (int i = 2; i < tsize; ++i) {
        mont_mul<S, G>(cur, cur, tbl, n, n0inv);
        lds_put<S, G>(tbl + (i - 1) * Ly::WORDS, cur);
    }
    lds_sync();

    // exponent length, maximised over the wave
    uint32_t ebits = 0;
    if (use_exp) {
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int li = r * L + k;
            const uint32_t v = li < elimbs ? ep[li] : 0u;
            if (v) ebits = (uint32_t)(32 * li + 32 - __clz(v));
        }
    }
    const uint32_t maxbits = wave_max(ebits);
    const int nwin = (int)((maxbits + (uint32_t)w - 1) / (uint32_t)w);

#pragma unroll
    for (int k = 0; k < L; ++k) A[k] = one[k];
    if (nwin == 0) return;

    uint32_t d = use_exp ? exp_digit(ep, elimbs, (nwin - 1) * w, w) : 0u;
    {
        uint32_t t[L];
        lds_get<S, G>(t, tbl + ((d ? d : 1u) - 1) * Ly::WORDS, g);
#pragma unroll
        for (int k = 0; k < L; ++k) A[k] = d ? t[k] : A[k];
    }
    for (int win = nwin - 2; win >= 0; --win) {
        d = use_exp ? exp_digit(ep, elimbs, win * w, w) : 0u;
        for (int s = 0; s < w; ++s) mont_sqr_lds<S, G>(A, abuf, n, n0inv);
        if (__ballot(d != 0u)) {
            uint32_t t[L];
            mont_mul<S, G>(t, A, tbl + ((d ? d : 1u) - 1) * Ly::WORDS, n, n0inv);
#pragma unroll
            for (int k = 0; k < L; ++k) A[k] = d ? t[k] : A[k];
        }
    }
}

// A = A * R^-1 mod n (leave Montgomery form).
template <int S, int G>
__device__ __forceinline__ void from_mont(uint32_t (&A)[S / G], uint32_t *abuf, const uint32_t (&n)[S / G],
                                          uint32_t n0inv)
{
    constexpr int L = S / G;
    uint32_t u[L];
#pragma unroll
    for (int k = 0; k < L; ++k) u[k] = (grp_lane<G>() == 0 && k == 0) ? 1u : 0u;
    mont_mul_reg<S, G>(A, A, u, abuf, n, n0inv);
}

// ---- out[i] = base[i]^exp[i] mod mod[i] --------------------------------
template <int S, int G>
__global__ __launch_bounds__(64) void k_modexp(const uint32_t *__restrict__ base,
                                               const uint32_t *__restrict__ exp,
                                               const uint32_t *__restrict__ mod,
                                               uint32_t *out, unsigned long long count, int limbs, int w,
                                               unsigned long long *errs)
{
    constexpr int L = S / G, NG = 64 / G;
    uint32_t *lds = reinterpret_cast<uint32_t *>(rsagpu_lds);
    const int g = grp_index<G>(), r = grp_lane<G>();
    const unsigned long long msg = (unsigned long long)blockIdx.x * NG + g;
    const bool live = msg < count;
    const size_t off = live ? (size_t)msg * (size_t)limbs : 0;

    uint32_t n[L], x[L];
    load_limbs<S, G>(n, mod + off, limbs, live);
    load_limbs<S, G>(x, base + off, limbs, live);
    const uint32_t n0 = grp_bcast<G>(n[0], 0);
    const uint32_t bl = grp_bitlen<S, G>(n);
    const bool valid = live && (n0 & 1u) && bl > 1;
    const uint32_t n0inv = neg_inv32(n0 | 1u);

    uint32_t one[L], r2[L], xt[L], A[L];
    mont_setup<S, G>(one, r2, n, n0inv, valid, lds);
    mont_mul_reg<S, G>(xt, x, r2, lds, n, n0inv);
    group_modexp<S, G>(A, xt, exp + off, limbs, valid, n, n0inv, one, lds, w);
    from_mont<S, G>(A, lds, n, n0inv);

    store_limbs<S, G>(out + off, A, limbs, live, valid);
    if (live && r == 0 && !valid && bl != 1) atomicAdd(errs, 1ull);
}

// ---- CRT decryption ------------------------------------------------------
//
// Groups come in pairs: even group = the half modulo p, odd group = modulo q
// of the same message; H is the (padded) width of p and q, hl their actual
// limb count, and the message c and result have 2*hl limbs.
template <int H, int G>
__global__ __launch_bounds__(64) void k_crt(const uint32_t *__restrict__ c, const uint32_t *__restrict__ p,
                                            const uint32_t *__restrict__ q, const uint32_t *__restrict__ dp,
                                            const uint32_t *__restrict__ dq, const uint32_t *__restrict__ qinv,
                                            uint32_t *out, unsigned long long count, int hl, int w,
                                            unsigned long long *errs)
{
    constexpr int L = H / G, NG = 64 / G;
    static_assert(NG >= 2, "a wave holds at least one pair of groups");
    uint32_t *lds = reinterpret_cast<uint32_t *>(rsagpu_lds);
    const int g = grp_index<G>(), r = grp_lane<G>();
    const int half = g & 1;
    const unsigned long long msg = (unsigned long long)blockIdx.x * (NG / 2) + (g >> 1);
    const bool live = msg < count;
    const size_t hoff = live ? (size_t)msg * (size_t)hl : 0;
    const size_t foff = 2 * hoff;

    uint32_t n[L], clo[L], chi[L], other[L];
    load_limbs<H, G>(n, (half ? q : p) + hoff, hl, live);
    load_limbs<H, G>(other, (half ? p : q) + hoff, hl, live);   // p-groups need q
    load_limbs<H, G>(clo, c + foff, hl, live);
    load_limbs<H, G>(chi, c + foff + hl, hl, live);
    const uint32_t n0 = grp_bcast<G>(n[0], 0);
    const uint32_t bl = grp_bitlen<H, G>(n);
    bool valid = live && (n0 & 1u) && bl > 1;
    {   // p > q, evaluated by every group and used by the p-groups
        uint32_t d[L];
        const uint32_t lt = grp_sub<H, G>(d, n, other);
        bool nz = false;
#pragma unroll
        for (int k = 0; k < L; ++k) nz = nz || d[k] != 0u;
        const bool gt = !lt && grp_any<G>(nz);
        valid = valid && (half || gt);
    }
    {   // a pair is valid only if both of its groups are
        const unsigned pbase = (lane_id() / (2 * G)) * (2 * G);
        const uint64_t pmask = (2 * G == 64) ? ~0ull : (((1ull << (2 * G)) - 1) << pbase);
        const bool bad = (__ballot(!valid) & pmask) != 0;
        valid = valid && !bad;
    }
    const uint32_t n0inv = neg_inv32(n0 | 1u);

    uint32_t one[L], r2[L], k3[L], y[L];
    mont_setup<H, G>(one, r2, n, n0inv, valid, lds);
    // y = 2^(32 hl) * R mod n: r2 when hl == H, else one doubled 32*hl times
#pragma unroll
    for (int k = 0; k < L; ++k) y[k] = (hl == H) ? r2[k] : one[k];
    if (hl != H)
        for (int t = 0; t < 32 * hl; ++t) grp_dbl_mod<H, G>(y, n);
    mont_mul_reg<H, G>(k3, y, r2, lds, n, n0inv);          // 2^(32 hl) * R^2 mod n

    // xt = c * R mod n = c_lo * R + c_hi * 2^(32 hl) * R
    uint32_t xt[L], t2[L];
    mont_mul_reg<H, G>(xt, clo, r2, lds, n, n0inv);
    mont_mul_reg<H, G>(t2, chi, k3, lds, n, n0inv);
    grp_add_mod<H, G>(xt, t2, n);

    uint32_t A[L];
    group_modexp<H, G>(A, xt, (half ? dq : dp) + hoff, hl, valid, n, n0inv, one, lds, w);
    from_mont<H, G>(A, lds, n, n0inv);

    // Garner: h = qinv * (m_p - m_q) mod p, m = m_q + h * q  (on the p-group)
    uint32_t mq[L], qv[L], hh[L];
    lds_sync();
    lds_put<H, G>(lds, A);
    lds_sync();
    lds_get<H, G>(mq, lds, g ^ 1);
    grp_sub_mod<H, G>(A, mq, n);                            // delta = m_p - m_q mod p
    load_limbs<H, G>(qv, qinv + hoff, hl, live && !half);
    mont_mul_reg<H, G>(qv, qv, r2, lds, n, n0inv);          // qinv * R mod p
    mont_mul_reg<H, G>(hh, A, qv, lds, n, n0inv);           // delta * qinv mod p
    lds_sync();
    lds_put<H, G>(lds, hh);
    lds_sync();
    const int full = 2 * hl;
    uint32_t *o = out + foff;
    const bool write = live && !half;
    auto sink = [&](int i, uint32_t v) {
        if (write && r == 0 && i < full) o[i] = valid ? v : 0u;
    };
    uint32_t high[L];
    mul_wide<H, G>(high, mq, other, lds, sink);
    if (write) {
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int li = H + r * L + k;
            if (li < full) o[li] = valid ? high[k] : 0u;
        }
    }
    if (write && r == 0 && !valid) atomicAdd(errs, 1ull);
}

}  // namespace rsagpu
