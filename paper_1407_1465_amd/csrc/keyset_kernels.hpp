// Resident-key kernels: Montgomery-constant setup for a key, and persistent
// per-bucket kernels that run a batch of operation descriptors.
//
// A key is held on the device as its raw 32-bit-word material (n, e, p, q,
// dp, dq, qinv) plus, for each limb radix the library computes in, the
// Montgomery constants of m = n, p and q stored as the kernel's limbs:
// one = R mod m and r2 = R^2 mod m for all three, r3 = R^3 mod m for p and q
// (CRT entry of a full-width ciphertext), and qinv * R mod p (Garner's
// multiplier in Montgomery form).  They are computed once when the key is
// added, so an operation starts directly with its exponentiation.
//
// Operations are grouped on the device into buckets of one (width class,
// kind), each ordered by key; each bucket is served by a persistent kernel
// whose workgroups claim a chunk of operations at a time from an atomic
// counter until the bucket is empty.
#pragma once

#include "modexp_kernels.hpp"

namespace rsagpu {

// Constants of one modulus m in one radix, S limbs each: one = R mod m,
// r2 = R^2 mod m, r3 = R^3 mod m and xr = x * R mod m for a multiplier x given
// at setup.  r3 and xr are null where no kernel needs them.
struct ModConsts {
    uint32_t *one;
    uint32_t *r2;
    uint32_t *r3;
    uint32_t *xr;
};

// Device view of one resident key.
struct KeyDev {
    int cls;                  // width class index
    int words;                // 32-bit words of n
    int hwords;               // 32-bit words of p and q
    int pad;
    const uint32_t *n, *e, *p, *q, *dp, *dq, *qinv;
    ModConsts cn[2], cp[2], cq[2];     // [0]: radix 2^32, [1]: radix 2^29
};

// One operation descriptor (layout shared with include/rsagpu.h rsa_op).
struct OpDesc {
    uint32_t kind;            // 0: in^e mod n, 1: CRT decryption
    int32_t key_id;
    unsigned long long in_off, out_off;
};

template <int B>
__device__ __forceinline__ int radix_slot() { return B == 32 ? 0 : 1; }

// Loads limbs [r*L, r*L+L) of an S-limb array of kernel limbs.
template <int S, int G>
__device__ __forceinline__ void load_raw(uint32_t (&x)[S / G], const uint32_t *p, bool live)
{
    constexpr int L = S / G;
    const int r = grp_lane<G>();
#pragma unroll
    for (int k = 0; k < L; ++k) x[k] = live ? p[r * L + k] : 0u;
}

template <int S, int G>
__device__ __forceinline__ void store_raw(uint32_t *p, const uint32_t (&x)[S / G], bool live)
{
    constexpr int L = S / G;
    const int r = grp_lane<G>();
    if (!live) return;
#pragma unroll
    for (int k = 0; k < L; ++k) p[r * L + k] = x[k];
}

// Constants of `count` moduli (32-bit words each at mods[i]) in radix 2^B
// with S limbs, written to outs[i]; xr from the multiplier mults[i] (same word
// count, below the modulus) where outs[i].xr is set.  The caller validated
// the moduli.
template <int S, int G, int B>
__global__ __launch_bounds__(64) void k_setup(const uint32_t *const *mods, const uint32_t *const *mults,
                                              const int *words, ModConsts *outs, int count)
{
    using Ar = Arith<S, G, B>;
    constexpr int L = S / G, NG = 64 / G;
    uint32_t *lds = reinterpret_cast<uint32_t *>(rsagpu_lds);
    const int g = grp_index<G>();
    const int i = blockIdx.x * NG + g;
    const bool live = i < count;
    uint32_t n[L];
    Ar::load(n, live ? mods[i] : nullptr, live ? words[i] : 0, 0, live);
    const uint32_t n0 = grp_bcast0<G>(n[0]);
    const uint32_t bl = Ar::bitlen(n);
    const bool valid = live && (n0 & 1u) && bl > 1;
    const uint32_t n0inv = Ar::n0inv(n0 | 1u);
    uint32_t one[L], r2[L], t[L];
    mont_setup<S, G, B>(one, r2, n, n0inv, valid, lds);
    const ModConsts oc = live ? outs[i] : ModConsts{nullptr, nullptr, nullptr, nullptr};
    store_raw<S, G>(oc.one, one, live);
    store_raw<S, G>(oc.r2, r2, live);
    mont_mul_reg<S, G, B>(t, r2, r2, lds, n, n0inv);           // R^3 mod m
    store_raw<S, G>(oc.r3, t, live && oc.r3);
    const bool want_x = live && oc.xr && mults[i];
    uint32_t x[L];
    Ar::load(x, want_x ? mults[i] : nullptr, want_x ? words[i] : 0, 0, want_x);
    mont_mul_reg<S, G, B>(t, x, r2, lds, n, n0inv);            // x * R mod m
    store_raw<S, G>(oc.xr, t, want_x);
}

// Claims the next chunk of `n` operations of a bucket for this wave.
__device__ __forceinline__ unsigned claim(unsigned *counter, unsigned n)
{
    unsigned base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, n);
    return (unsigned)__builtin_amdgcn_readfirstlane((int)base);
}

// Bucket of encryptions (in^e mod n) for keys of one width class: S limbs of
// radix 2^B hold n.
template <int S, int G, int B>
__global__ __launch_bounds__(64) RSAGPU_EXP_OCC(S / G) void k_ops_enc(const KeyDev *__restrict__ keys, const OpDesc *__restrict__ ops,
                                                const unsigned *__restrict__ list, const unsigned *count_p,
                                                unsigned *counter, const uint32_t *__restrict__ in_pool,
                                                uint32_t *out_pool, int w, int urgent)
{
    using Ar = Arith<S, G, B>;
    constexpr int L = S / G, NG = 64 / G;
    constexpr bool OWN = B != 32 && !standard_s29(S);     // constants not in the keyset's limb count
    uint32_t *lds = reinterpret_cast<uint32_t *>(rsagpu_lds);
    const int g = grp_index<G>();
    const unsigned count = *count_p;
    if (urgent) __builtin_amdgcn_s_setprio(2);
    for (;;) {
        const unsigned base = claim(counter, NG);
        if (base >= count) break;                     // wave-uniform exit
        const unsigned idx = base + g;
        const unsigned at = idx < count ? list[idx] : kOrderHole;
        const bool live = at != kOrderHole;
        const OpDesc op = ops[live ? at : list[base]];   // a wave's first entry is never a hole
        const KeyDev &k = keys[op.key_id];
        const ModConsts &mc = k.cn[radix_slot<B>()];
        uint32_t n[L], x[L], one[L], r2[L], xt[L], A[L];
        Ar::load(n, k.n, k.words, 0, live);
        Ar::load(x, in_pool + op.in_off, k.words, 0, live);
        const uint32_t n0inv = Ar::n0inv(grp_bcast0<G>(n[0]) | 1u);
        if constexpr (OWN) {
            mont_setup<S, G, B>(one, r2, n, n0inv, live, lds);
        } else {
            load_raw<S, G>(one, mc.one, live);
            load_raw<S, G>(r2, mc.r2, live);
        }
        mont_mul_reg<S, G, B>(xt, x, r2, lds, n, n0inv);
        if (!group_modexp<S, G, B, true>(A, xt, k.e, k.words, live, n, n0inv, one, lds, w, x))
            from_mont<S, G, B>(A, lds, n, n0inv);
        store_words<S, G, B>(out_pool + op.out_off, A, k.words, live, true, lds);
    }
}

// Bucket of CRT decryptions for keys of one width class: H limbs of radix
// 2^B hold p and q.  A workgroup of P pairs of waves (P = 1, or 2 in the
// CRT buckets of a bulk batch where the LDS holds them, see crt_pairs)
// claims P * NG operations at a time (NG = 64 / G), each pair a
// run of NG of them: the pair's wave 0 takes their halves modulo p, its wave
// 1 those modulo q, one operation per lane group, so a run of one key's
// operations (the bucket lists are ordered by key, each key's run starting a
// run of NG where that fits) gives each wave a single exponent; entries
// kOrderHole (the rest of such a run) are skipped.  m_q reaches the pair's
// wave 0 through its wave 1's LDS region; wave 0 recombines and stores.
template <int H, int G, int B, int P>
__global__ __launch_bounds__(128 * P) void k_ops_crt(const KeyDev *__restrict__ keys, const OpDesc *__restrict__ ops,
                                                     const unsigned *__restrict__ list, const unsigned *count_p,
                                                     unsigned *counter, const uint32_t *__restrict__ in_pool,
                                                     uint32_t *out_pool, int w, int urgent)
{
    using Ar = Arith<H, G, B>;
    using Ly = Layout<H, G>;
    constexpr int L = H / G, NG = 64 / G;
    constexpr bool OWN = B != 32 && !standard_s29(H);     // constants not in the keyset's limb count
    __shared__ unsigned chunk;
    const int wave = (int)(threadIdx.x >> 6), pair = wave >> 1, half = wave & 1;
    const size_t region = (size_t)lds_entries(B, G, w) * Ly::WORDS;
    uint32_t *lds = reinterpret_cast<uint32_t *>(rsagpu_lds) + wave * region;
    uint32_t *qlds = reinterpret_cast<uint32_t *>(rsagpu_lds) + (2 * pair + 1) * region;   // the pair's wave 1
    const int g = grp_index<G>(), r = grp_lane<G>();
    const unsigned count = *count_p;
    if (urgent) __builtin_amdgcn_s_setprio(2);
    for (;;) {
        // The wave 0s reach this barrier after Garner has read the previous
        // chunk's m_q, and every wave reads `chunk` before the barrier below:
        // neither the claim nor a wave 1's next use of its region overtakes.
        if (threadIdx.x == 0) chunk = atomicAdd(counter, (unsigned)(P * NG));
        __syncthreads();
        const unsigned base = chunk;
        if (base >= count) break;                     // the same for every wave
        const unsigned idx = base + pair * NG + g;
        const unsigned at = idx < count ? list[idx] : kOrderHole;
        const bool live = at != kOrderHole;
        const OpDesc op = ops[live ? at : list[base]];   // a wave's first entry is never a hole
        const KeyDev &k = keys[op.key_id];
        const int hl = k.hwords, full = 2 * hl;
        const ModConsts &mc = half ? k.cq[radix_slot<B>()] : k.cp[radix_slot<B>()];
        uint32_t n[L], clo[L], chi[L], one[L], rk[L];
        Ar::load(n, half ? k.q : k.p, hl, 0, live);
        Ar::load(clo, in_pool + op.in_off, full, 0, live);
        Ar::load(chi, in_pool + op.in_off, full, B * H, live);
        const uint32_t n0inv = Ar::n0inv(grp_bcast0<G>(n[0]) | 1u);
        // xt = c * R mod m = c_lo * R^2 * R^-1 + c_hi * R^3 * R^-1  (c = c_lo + c_hi * R)
        uint32_t xt[L], t2[L], r2[L];
        if constexpr (OWN) {
            mont_setup<H, G, B>(one, r2, n, n0inv, live, lds);
            mont_mul_reg<H, G, B>(xt, clo, r2, lds, n, n0inv);
            mont_mul_reg<H, G, B>(rk, r2, r2, lds, n, n0inv);        // R^3 mod m
            mont_mul_reg<H, G, B>(t2, chi, rk, lds, n, n0inv);
        } else {
            load_raw<H, G>(rk, mc.r2, live);
            mont_mul_reg<H, G, B>(xt, clo, rk, lds, n, n0inv);
            load_raw<H, G>(rk, mc.r3, live);
            mont_mul_reg<H, G, B>(t2, chi, rk, lds, n, n0inv);
            load_raw<H, G>(one, mc.one, live);
        }
        {
            const uint32_t ovf = Ar::add(xt, t2);
            Ar::cond_sub(xt, ovf, n);
        }
        uint32_t A[L];
        group_modexp<H, G, B>(A, xt, half ? k.dq : k.dp, hl, live, n, n0inv, one, lds, w, xt);
        from_mont<H, G, B>(A, lds, n, n0inv);

        if (half) {
            lds_sync();
            lds_put<H, G>(qlds, A);
        }
        __syncthreads();
        if (half) continue;

        // Garner: h = qinv * (m_p - m_q) mod p, m = m_q + h * q
        uint32_t mq[L], qv[L], hh[L];
        lds_get<H, G>(mq, qlds, g);
        {   // delta = m_p - m_q mod p  (m_q < q < p)
            uint32_t d[L], e[L];
            const uint32_t neg = Ar::sub(d, A, mq);
#pragma unroll
            for (int j = 0; j < L; ++j) e[j] = d[j];
            Ar::add(e, n);
#pragma unroll
            for (int j = 0; j < L; ++j) A[j] = neg ? e[j] : d[j];
        }
        if constexpr (OWN) {
            Ar::load(qv, k.qinv, hl, 0, live);
            mont_mul_reg<H, G, B>(qv, qv, r2, lds, n, n0inv);     // qinv * R mod p
        } else {
            load_raw<H, G>(qv, k.cp[radix_slot<B>()].xr, live);  // qinv * R mod p
        }
        mont_mul_reg<H, G, B>(hh, A, qv, lds, n, n0inv);
        lds_sync();
        lds_put<H, G>(lds, hh);
        lds_sync();
        uint32_t *stage = lds + Ly::WORDS + g * (2 * H);
        auto sink = [&](int i, uint32_t v) {
            if (r == 0) stage[i] = v;
        };
        uint32_t high[L], qn[L];
        Ar::load(qn, k.q, hl, 0, live);
        Ar::mul_wide(high, mq, qn, lds, sink);
#pragma unroll
        for (int j = 0; j < L; ++j) stage[H + r * L + j] = high[j];
        lds_sync();
        if (live) {
            uint32_t *o = out_pool + op.out_off;
            if constexpr (B == 32) {
                for (int wd = r; wd < full; wd += G) o[wd] = stage[wd];
            } else {
                for (int wd = r; wd < full; wd += G) o[wd] = rword<B>(stage, 2 * H, wd);
            }
        }
        lds_sync();
    }
}

}  // namespace rsagpu
