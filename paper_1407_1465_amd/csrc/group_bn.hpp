// Lane-group multi-precision arithmetic for CDNA4 (gfx950, wave64).
//
// One big integer of S 32-bit limbs is spread over a group of G consecutive
// lanes of a wavefront; lane r of the group holds limbs [r*L, r*L + L), with
// L = S / G.  A wave therefore works on NG = 64 / G integers at once.  Every
// function here is called by all 64 lanes of the wave in lockstep; lanes of
// different groups work on different integers.
//
// Montgomery multiplication (Montgomery 1985) is organised as coarsely
// integrated operand scanning (CIOS, Koc, Acar and Kaliski 1996): for each
// limb b_i of the multiplier, add a*b_i, derive m = t_0 * (-n^-1) mod 2^32,
// add m*n and drop the (now zero) bottom limb.  The distribution over lanes
// and the carry handling are this library's own:
//
//   * each limb position of the running sum t is a 96-bit accumulator
//     (a 64-bit register pair plus a carry-count word), so every 32x32-bit
//     product costs one v_mad_u64_u32 (carry-out to VCC) and one
//     v_addc_co_u32 - no carry chain runs along the limbs inside the loop;
//   * after each step every lane folds the high 64 bits of its bottom
//     position into the next position, so the word that moves to the lane
//     below is a plain 32-bit value; lane 0 of the group drops it (it is the
//     zero word of the Montgomery shift);
//   * limb positions rotate through the registers (position j of step k is
//     register (j + k) mod L), so the shift by one limb costs no moves;
//   * carries are resolved once per product, across lanes, with one wave
//     ballot for "generate" and one for "propagate" and a 64-bit scalar add
//     (the carry-lookahead identity carries = (A + B) ^ A ^ B).
//
// The multiplier b is read from LDS (group-uniform addresses, so a broadcast
// within the group) or, for groups of 1, 2 or 4 lanes, broadcast from the
// group's own registers by DPP (mont_mul_regs); the multiplicand a and the
// modulus n sit in VGPRs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsagpu {

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

template <int G>
__device__ __forceinline__ unsigned grp_lane() { return lane_id() & (G - 1); }

template <int G>
__device__ __forceinline__ unsigned grp_index() { return lane_id() / G; }

// Bit mask of the lanes that are the top lane of their group.
template <int G>
__device__ __forceinline__ constexpr uint64_t top_lanes_mask()
{
    uint64_t m = 0;
    for (int l = G - 1; l < 64; l += G) m |= 1ull << l;
    return m;
}

// ---- cross-lane moves inside a group -----------------------------------
//
// Groups of up to 16 lanes never straddle a DPP row, so the moves below are
// DPP data movements (no LDS round trip): quad_perm for groups of 2 and 4,
// row shifts with bank masks for 8 and 16, and for the broadcast of any lane
// of a 16-lane group the row broadcast that CDNA3/4 DPP provides.

template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, BANK_MASK, false);
}

// Every lane written; a lane whose source is outside its row reads 0
// (bound_ctrl).  No previous value is involved, so the destination needs no
// initialising move.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp0(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

enum : int {
    DPP_QP_0000 = 0x00,      // quad_perm [0,0,0,0]
    DPP_QP_0022 = 0xA0,      // quad_perm [0,0,2,2]
    DPP_QP_1230 = 0x39,      // quad_perm [1,2,3,0]
    DPP_QP_1032 = 0xB1,      // quad_perm [1,0,3,2]
    DPP_QP_1133 = 0xF5,      // quad_perm [1,1,3,3]
    DPP_ROW_SHL1 = 0x101,    // lane i <- lane i+1 within a row of 16
    DPP_ROW_SHR1 = 0x111,    // lane i <- lane i-1 within a row of 16
    DPP_ROW_SHR4 = 0x114,
    DPP_ROW_NEWBCAST0 = 0x150,  // every lane of a row of 16 <- the row's lane 0 (+K: lane K)
};

// Value of lane 0 of this lane's group.
template <int G>
__device__ __forceinline__ uint32_t grp_bcast0(uint32_t v)
{
    if constexpr (G == 1) return v;
    else if constexpr (G == 2) return dpp0<DPP_QP_0022>(v);
    else if constexpr (G == 4) return dpp0<DPP_QP_0000>(v);
    else if constexpr (G == 8) {
        const uint32_t q = dpp0<DPP_QP_0000>(v);
        return dpp<DPP_ROW_SHR4, 0xF, 0xA>(q, q);           // banks 1, 3 take banks 0, 2
    } else if constexpr (G == 16) return dpp0<DPP_ROW_NEWBCAST0>(v);
    else return (uint32_t)__shfl((int)v, 0, G);
}

// grp_bcast0(v) & mask, with the mask applied right after the first
// (full-write) lane move so that the two fold into one DPP-modified AND
// (mask in a VGPR); the later bank-masked moves copy the masked value.
template <int G>
__device__ __forceinline__ uint32_t grp_bcast0_and(uint32_t v, uint32_t mask)
{
    if constexpr (G == 1) return v & mask;
    else if constexpr (G == 2 || G == 4) return grp_bcast0<G>(v) & mask;
    else if constexpr (G == 8) {
        const uint32_t q = dpp0<DPP_QP_0000>(v) & mask;
        return dpp<DPP_ROW_SHR4, 0xF, 0xA>(q, q);
    } else if constexpr (G == 16) {
        return dpp0<DPP_ROW_NEWBCAST0>(v) & mask;
    } else return grp_bcast0<G>(v) & mask;
}

// Value of lane K of this lane's group (G = 1, 2, 4 or 16: one DPP quad
// permute, or for 16 lanes the row broadcast of lane K).
template <int G, int K>
__device__ __forceinline__ uint32_t grp_bcast_lane(uint32_t v)
{
    static_assert(G == 1 || G == 2 || G == 4 || G == 16, "quad permutes or a row broadcast only");
    static_assert(K >= 0 && K < G, "lane of the group");
    if constexpr (G == 1) return v;
    else if constexpr (G == 2) return dpp0<K == 0 ? DPP_QP_0022 : DPP_QP_1133>(v);
    else if constexpr (G == 4) return dpp0<K * 0x55>(v);    // quad_perm [K, K, K, K]
    else return dpp0<DPP_ROW_NEWBCAST0 + K>(v);           // row_newbcast:K
}

// grp_rot_down(v) & mask with the mask folded into the row shift for 8 and
// 16 lanes (the same lane-0-is-zero condition as grp_rot_down).
template <int G>
__device__ __forceinline__ uint32_t grp_rot_down_and(uint32_t v, uint32_t mask);

// Lane r receives lane (r+1) mod G of its group.  Used where the group's
// lane 0 holds zero, so the top lane receives zero (groups of 8 need an
// explicit zero for the one top lane that a row shift does not reach).
template <int G>
__device__ __forceinline__ uint32_t grp_rot_down(uint32_t v)
{
    if constexpr (G == 1) return 0;
    else if constexpr (G == 2) return dpp0<DPP_QP_1032>(v);
    else if constexpr (G == 4) return dpp0<DPP_QP_1230>(v);
    else if constexpr (G == 8) {
        const uint32_t u = dpp0<DPP_ROW_SHL1>(v);
        return (lane_id() & 7) == 7 ? 0u : u;
    } else if constexpr (G == 16) return dpp0<DPP_ROW_SHL1>(v);
    else {
        const uint32_t u = (uint32_t)__shfl_down((int)v, 1, G);
        return (lane_id() & (G - 1)) == G - 1 ? 0u : u;
    }
}

template <int G>
__device__ __forceinline__ uint32_t grp_rot_down_and(uint32_t v, uint32_t mask)
{
    if constexpr (G == 8) {
        const uint32_t u = dpp0<DPP_ROW_SHL1>(v) & mask;
        return (lane_id() & 7) == 7 ? 0u : u;
    } else if constexpr (G == 16) {
        return dpp0<DPP_ROW_SHL1>(v) & mask;
    } else {
        return grp_rot_down<G>(v) & mask;
    }
}

// Lane r receives lane r+1's value; the group's top lane receives 0.
template <int G>
__device__ __forceinline__ uint32_t grp_from_above(uint32_t v)
{
    if constexpr (G == 1) return 0;
    else {
        const uint32_t u = (G <= 16) ? dpp0<DPP_ROW_SHL1>(v)
                                     : (uint32_t)__shfl_down((int)v, 1, G);
        return (lane_id() & (G - 1)) == G - 1 ? 0u : u;
    }
}

// Lane r receives lane r-1's value; the group's lane 0 receives 0.
template <int G>
__device__ __forceinline__ uint32_t grp_from_below(uint32_t v)
{
    if constexpr (G == 1) return 0;
    else {
        const uint32_t u = (G <= 16) ? dpp0<DPP_ROW_SHR1>(v)
                                     : (uint32_t)__shfl_up((int)v, 1, G);
        return (lane_id() & (G - 1)) == 0 ? 0u : u;
    }
}

// Carry (or borrow) into each lane of a multi-lane addition.  `gen`: this
// lane's own limbs produced a carry out; `prop`: an incoming carry would run
// through all of this lane's limbs.  Carries never cross a group boundary:
// what leaves a group's top lane is that group's overflow, handled by the
// caller.
template <int G>
__device__ __forceinline__ uint32_t grp_carry_in(bool gen, bool prop)
{
    if constexpr (G == 1) return 0;
    else {
        const uint64_t keep = ~top_lanes_mask<G>();
        const uint64_t gm = __ballot(gen) & keep;
        const uint64_t pm = __ballot(prop) & keep;
        const uint64_t a = gm | pm;
        const uint64_t c = (a + gm) ^ a ^ gm;
        return (uint32_t)(c >> lane_id()) & 1u;
    }
}

// Every lane of a group gets the flag of its group's top lane.
template <int G>
__device__ __forceinline__ bool grp_top_flag(bool f)
{
    if constexpr (G == 1) return f;
    else {
        const uint64_t m = __ballot(f && grp_lane<G>() == G - 1);
        const unsigned top = (lane_id() & ~(unsigned)(G - 1)) + (G - 1);
        return (m >> top) & 1ull;
    }
}

// True in every lane of a group when the predicate holds in any lane of it.
template <int G>
__device__ __forceinline__ bool grp_any(bool f)
{
    if constexpr (G == 1) return f;
    else {
        const uint64_t m = __ballot(f);
        const unsigned base = lane_id() & ~(unsigned)(G - 1);
        const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1) << base);
        return (m & gmask) != 0;
    }
}

template <int G>
__device__ __forceinline__ uint32_t grp_max(uint32_t v)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        uint32_t u = (uint32_t)__shfl_xor((int)v, o, G);
        v = u > v ? u : v;
    }
    return v;
}

// c held in a VGPR rather than as an instruction literal, so that a DPP lane
// move feeding an operation with c can fold into one DPP-modified VOP2
// instruction (their second operand must be a VGPR).
__device__ __forceinline__ uint32_t vgpr_const(uint32_t c)
{
    uint32_t v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "i"(c));
    return v;
}

// The first active lane's value of a pointer (wave-uniform from here on).
__device__ __forceinline__ const uint32_t *first_lane_ptr(const uint32_t *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (const uint32_t *)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = (uint32_t)__shfl_xor((int)v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

// ---- single-lane limb helpers --------------------------------------------

// {acc} += x*y as a 64-bit sum; the carry out of bit 63 is added to hi.
__device__ __forceinline__ void mac(uint64_t &acc, uint32_t &hi, uint32_t x, uint32_t y)
{
    asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t"
        "v_addc_co_u32 %1, vcc, 0, %1, vcc"
        : "+v"(acc), "+v"(hi)
        : "v"(x), "v"(y)
        : "vcc");
}

// Two independent macs; their carries go through two distinct SGPR pairs so
// the second product issues while the first carry is still in flight.
__device__ __forceinline__ void mac2(uint64_t &acc0, uint32_t &hi0, uint32_t x0, uint64_t &acc1, uint32_t &hi1,
                                     uint32_t x1, uint32_t y)
{
    uint64_t c0, c1;
    asm("v_mad_u64_u32 %0, %4, %6, %8, %0\n\t"
        "v_mad_u64_u32 %1, %5, %7, %8, %1\n\t"
        "v_addc_co_u32_e64 %2, %4, 0, %2, %4\n\t"
        "v_addc_co_u32_e64 %3, %5, 0, %3, %5"
        : "+v"(acc0), "+v"(acc1), "+v"(hi0), "+v"(hi1), "=&s"(c0), "=&s"(c1)
        : "v"(x0), "v"(x1), "v"(y));
}

// Row update: acc[(j + k) % L] += x[j] * y for all j.
template <int L>
__device__ __forceinline__ void mac_row(uint64_t (&acc)[L], uint32_t (&hi)[L], const uint32_t (&x)[L], uint32_t y,
                                        int k)
{
#pragma unroll
    for (int j = 0; j + 1 < L; j += 2)
        mac2(acc[(j + k) % L], hi[(j + k) % L], x[j], acc[(j + 1 + k) % L], hi[(j + 1 + k) % L], x[j + 1], y);
    if constexpr (L % 2 == 1) mac(acc[(L - 1 + k) % L], hi[(L - 1 + k) % L], x[L - 1], y);
}

// (acc, hi) += x  where x is a 64-bit value at the same weight as acc.
__device__ __forceinline__ void add96(uint64_t &acc, uint32_t &hi, uint32_t xlo, uint32_t xhi)
{
    unsigned c0, c1, c2;
    const uint32_t a0 = __builtin_addc((uint32_t)acc, xlo, 0u, &c0);
    const uint32_t a1 = __builtin_addc((uint32_t)(acc >> 32), xhi, c0, &c1);
    hi = __builtin_addc(hi, 0u, c1, &c2);
    acc = ((uint64_t)a1 << 32) | a0;
}

// -n0^-1 mod 2^32 for odd n0 (Newton-Hensel lifting: x <- x(2 - n0 x)
// doubles the number of correct low bits; n0 itself is correct to 3 bits).
__device__ __forceinline__ uint32_t neg_inv32(uint32_t n0)
{
    uint32_t x = n0;
#pragma unroll
    for (int i = 0; i < 4; ++i) x *= 2u - n0 * x;
    return 0u - x;
}

// ---- LDS operand layout ---------------------------------------------------
//
// An operand buffer holds one S-limb integer for each of the NG groups of a
// wave.  Limb i of group g is at word ((i / V) * NG + g) * V + i % V, so a
// group reads V consecutive limbs with one vector load and, in every step,
// the NG groups of a wave read NG different banks.
template <int S, int G>
struct Layout {
    static constexpr int L = S / G;
    static constexpr int NG = 64 / G;
    static constexpr int V = (L % 4 == 0) ? 4 : ((L % 2 == 0) ? 2 : 1);
    static constexpr int WORDS = S * NG;   // words of one operand buffer
    __device__ static constexpr int at(int limb, int g) { return ((limb / V) * NG + g) * V + (limb % V); }
};

template <int V>
struct VecT;
template <> struct VecT<1> { typedef uint32_t T; };
template <> struct VecT<2> { typedef uint2 T; };
template <> struct VecT<4> { typedef uint4 T; };

// Each lane stores its L limbs of x into the group's slot of buffer buf.
template <int S, int G>
__device__ __forceinline__ void lds_put(uint32_t *buf, const uint32_t (&x)[S / G])
{
    using Ly = Layout<S, G>;
    const int g = grp_index<G>(), r = grp_lane<G>();
#pragma unroll
    for (int k = 0; k < Ly::L; k += Ly::V) {
        typename VecT<Ly::V>::T v;
        uint32_t *pv = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
        for (int u = 0; u < Ly::V; ++u) pv[u] = x[k + u];
        *reinterpret_cast<typename VecT<Ly::V>::T *>(buf + Ly::at(r * Ly::L + k, g)) = v;
    }
}

// Each lane loads its L limbs of group slot gs of buffer buf.
template <int S, int G>
__device__ __forceinline__ void lds_get(uint32_t (&x)[S / G], const uint32_t *buf, int gs)
{
    using Ly = Layout<S, G>;
    const int r = grp_lane<G>();
#pragma unroll
    for (int k = 0; k < Ly::L; k += Ly::V) {
        typename VecT<Ly::V>::T v =
            *reinterpret_cast<const typename VecT<Ly::V>::T *>(buf + Ly::at(r * Ly::L + k, gs));
        const uint32_t *pv = reinterpret_cast<const uint32_t *>(&v);
#pragma unroll
        for (int u = 0; u < Ly::V; ++u) x[k + u] = pv[u];
    }
}

// Orders this wave's LDS traffic between its lanes.  Every wave works in an
// LDS region of its own, and one wave's LDS operations are performed in the
// order it issues them, so only the compiler has to be kept from moving
// accesses across this point (a wavefront-scope fence emits no wait).  Data
// exchanged between the waves of a workgroup needs __syncthreads().
__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- group-wide add / subtract / compare -------------------------------

// x += y over the group; returns the overflow bit in every lane of the group.
template <int S, int G>
__device__ __forceinline__ uint32_t grp_add(uint32_t (&x)[S / G], const uint32_t (&y)[S / G])
{
    constexpr int L = S / G;
    unsigned c = 0;
    uint32_t all = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < L; ++j) {
        x[j] = __builtin_addc(x[j], y[j], c, &c);
        all &= x[j];
    }
    const unsigned cin = grp_carry_in<G>(c != 0, all == 0xFFFFFFFFu);
    unsigned k = cin;
#pragma unroll
    for (int j = 0; j < L; ++j) x[j] = __builtin_addc(x[j], 0u, k, &k);
    return grp_top_flag<G>((c | k) != 0) ? 1u : 0u;
}

// d = x - y over the group; returns 1 in every lane of the group when x < y.
template <int S, int G>
__device__ __forceinline__ uint32_t grp_sub(uint32_t (&d)[S / G], const uint32_t (&x)[S / G],
                                            const uint32_t (&y)[S / G])
{
    constexpr int L = S / G;
    unsigned b = 0;
    uint32_t any = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
        d[j] = __builtin_subc(x[j], y[j], b, &b);
        any |= d[j];
    }
    const unsigned bin = grp_carry_in<G>(b != 0, any == 0u);
    unsigned k = bin;
#pragma unroll
    for (int j = 0; j < L; ++j) d[j] = __builtin_subc(d[j], 0u, k, &k);
    return grp_top_flag<G>((b | k) != 0) ? 1u : 0u;
}

// x = (x + top * 2^(32S)) mod n for x + top*2^(32S) < 2n; `top` is read from
// the group's top lane only (other lanes pass anything).
template <int S, int G>
__device__ __forceinline__ void grp_cond_sub(uint32_t (&x)[S / G], uint32_t top,
                                             const uint32_t (&n)[S / G])
{
    constexpr int L = S / G;
    uint32_t d[L];
    const uint32_t borrow = grp_sub<S, G>(d, x, n);
    const bool over = grp_top_flag<G>(top != 0);
    const bool take = over || !borrow;
#pragma unroll
    for (int j = 0; j < L; ++j) x[j] = take ? d[j] : x[j];
}

// x = 2x mod n for x < n.
template <int S, int G>
__device__ __forceinline__ void grp_dbl_mod(uint32_t (&x)[S / G], const uint32_t (&n)[S / G])
{
    constexpr int L = S / G;
    const uint32_t out = x[L - 1] >> 31;
    const uint32_t in = grp_from_below<G>(out);
#pragma unroll
    for (int j = L - 1; j > 0; --j) x[j] = (x[j] << 1) | (x[j - 1] >> 31);
    x[0] = (x[0] << 1) | in;
    grp_cond_sub<S, G>(x, out, n);
}

// Highest set bit + 1 of the group's integer (0 for zero), in every lane.
template <int S, int G>
__device__ __forceinline__ uint32_t grp_bitlen(const uint32_t (&x)[S / G])
{
    constexpr int L = S / G;
    uint32_t bl = 0;
#pragma unroll
    for (int j = 0; j < L; ++j)
        if (x[j]) bl = (uint32_t)(32 * (grp_lane<G>() * L + j) + 32 - __clz(x[j]));
    return grp_max<G>(bl);
}

// ---- normalisation of the redundant accumulator ------------------------

// Turns the L 96-bit positions of each lane into S normalised limbs plus the
// group's overflow (returned, meaningful in the top lane).  w receives the
// limbs.
template <int S, int G>
__device__ __forceinline__ uint32_t grp_normalise(uint32_t (&w)[S / G], const uint64_t (&acc)[S / G],
                                                  const uint32_t (&hi)[S / G])
{
    constexpr int L = S / G;
    static_assert(L >= 2, "at least two limbs per lane");
    // ripple inside the lane: position j is acc[j] + hi[j] * 2^64
    uint32_t clo = 0, chi = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
        unsigned c0, c1, c2;
        w[j] = __builtin_addc((uint32_t)acc[j], clo, 0u, &c0);
        clo = __builtin_addc((uint32_t)(acc[j] >> 32), chi, c0, &c1);
        chi = __builtin_addc(hi[j], 0u, c1, &c2);
    }
    // the 64-bit carry of each lane enters the lane above
    const uint32_t rlo = grp_from_below<G>(clo), rhi = grp_from_below<G>(chi);
    const bool top = grp_lane<G>() == G - 1;
    unsigned k;
    w[0] = __builtin_addc(w[0], rlo, 0u, &k);
    w[1] = __builtin_addc(w[1], rhi, k, &k);
#pragma unroll
    for (int j = 2; j < L; ++j) w[j] = __builtin_addc(w[j], 0u, k, &k);
    uint32_t all = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < L; ++j) all &= w[j];
    unsigned k2 = grp_carry_in<G>(k != 0, all == 0xFFFFFFFFu);
#pragma unroll
    for (int j = 0; j < L; ++j) w[j] = __builtin_addc(w[j], 0u, k2, &k2);
    // what leaves the group (meaningful in the top lane)
    return top ? (clo | chi | k | k2) : 0u;
}

// ---- Montgomery product -------------------------------------------------
//
// r = a * b * 2^(-32S) mod n, with a < 2^(32S) in registers, b < n in the
// group's slot of LDS buffer bbuf (or a < n and b < 2^(32S)), n odd.
// Mode Wide (used for the plain product of the CRT recombination): no
// reduction; the bottom limb of each step is handed to `sink` instead.
// The L CIOS steps of one block in radix 2^32 (96-bit positions acc:hi),
// multiplier limbs bv[0 .. L) already broadcast to the group.
template <int S, int G>
__device__ __forceinline__ void cios32_block(uint64_t (&acc)[S / G], uint32_t (&hi)[S / G],
                                             const uint32_t (&a)[S / G], const uint32_t (&bv)[S / G],
                                             const uint32_t (&n)[S / G], uint32_t n0inv)
{
    constexpr int L = S / G;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        // position j of this step lives in register (j + k) % L
        mac_row<L>(acc, hi, a, bv[k], k);
        const int p0 = k % L, p1 = (k + 1) % L;
        const uint32_t m = grp_bcast0<G>((uint32_t)acc[p0] * n0inv);
        mac_row<L>(acc, hi, n, m, k);
        add96(acc[p1], hi[p1], (uint32_t)(acc[p0] >> 32), hi[p0]);
        // the bottom word of the group's lane 0 is zero here, so a
        // rotation inside the group moves zero into the top lane
        acc[p0] = grp_rot_down<G>((uint32_t)acc[p0]);
        hi[p0] = 0;
    }
}

template <int S, int G>
__device__ __forceinline__ void mont_mul(uint32_t (&r)[S / G], const uint32_t (&a)[S / G],
                                         const uint32_t *bbuf, const uint32_t (&n)[S / G],
                                         uint32_t n0inv)
{
    using Ly = Layout<S, G>;
    constexpr int L = Ly::L, V = Ly::V;
    const int g = grp_index<G>();
    uint64_t acc[L];
    uint32_t hi[L];
#pragma unroll
    for (int j = 0; j < L; ++j) { acc[j] = 0; hi[j] = 0; }

    for (int i0 = 0; i0 < S; i0 += L) {
        uint32_t bv[L];
#pragma unroll
        for (int k = 0; k < L; k += V) {
            typename VecT<V>::T v = *reinterpret_cast<const typename VecT<V>::T *>(bbuf + Ly::at(i0 + k, g));
            const uint32_t *pv = reinterpret_cast<const uint32_t *>(&v);
#pragma unroll
            for (int u = 0; u < V; ++u) bv[k + u] = pv[u];
        }
        cios32_block<S, G>(acc, hi, a, bv, n, n0inv);
    }
    const uint32_t top = grp_normalise<S, G>(r, acc, hi);
    grp_cond_sub<S, G>(r, top, n);
}

// Blocks Q .. G-1 of a radix-2^32 product whose multiplier b is held in the
// group's registers like a: block Q takes limbs Q*L .. Q*L+L-1 (lane Q).
template <int S, int G, int Q>
struct Regs32Blocks {
    static __device__ __forceinline__ void run(uint64_t (&acc)[S / G], uint32_t (&hi)[S / G],
                                               const uint32_t (&a)[S / G], const uint32_t (&b)[S / G],
                                               const uint32_t (&n)[S / G], uint32_t n0inv)
    {
        if constexpr (Q < G) {
            constexpr int L = S / G;
            uint32_t bv[L];
#pragma unroll
            for (int k = 0; k < L; ++k) bv[k] = grp_bcast_lane<G, Q>(b[k]);
            cios32_block<S, G>(acc, hi, a, bv, n, n0inv);
            Regs32Blocks<S, G, Q + 1>::run(acc, hi, a, b, n, n0inv);
        }
    }
};

// mont_mul with the multiplier in the group's registers (G = 1, 2 or 4):
// no LDS round trip; r may alias a or b.
template <int S, int G>
__device__ __forceinline__ void mont_mul_regs(uint32_t (&r)[S / G], const uint32_t (&a)[S / G],
                                              const uint32_t (&b)[S / G], const uint32_t (&n)[S / G],
                                              uint32_t n0inv)
{
    constexpr int L = S / G;
    uint64_t acc[L];
    uint32_t hi[L];
#pragma unroll
    for (int j = 0; j < L; ++j) { acc[j] = 0; hi[j] = 0; }
    Regs32Blocks<S, G, 0>::run(acc, hi, a, b, n, n0inv);
    const uint32_t top = grp_normalise<S, G>(r, acc, hi);
    grp_cond_sub<S, G>(r, top, n);
}

// Plain product used by the CRT recombination:
//   (low, high) = init + a * b,   init < 2^(32S), a, b < 2^(32S)
// b in LDS.  The S low limbs are produced one per step; lane 0 of the group
// passes low limb i to sink(i, limb).  high receives the upper S limbs.
template <int S, int G, typename Sink>
__device__ __forceinline__ void mul_wide(uint32_t (&high)[S / G], const uint32_t (&init)[S / G],
                                         const uint32_t (&a)[S / G], const uint32_t *bbuf, Sink sink)
{
    using Ly = Layout<S, G>;
    constexpr int L = Ly::L, V = Ly::V;
    const int g = grp_index<G>();
    uint64_t acc[L];
    uint32_t hi[L];
#pragma unroll
    for (int j = 0; j < L; ++j) { acc[j] = init[j]; hi[j] = 0; }

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
            mac_row<L>(acc, hi, a, bv[k], k);
            const int p0 = k % L, p1 = (k + 1) % L;
            sink(i0 + k, (uint32_t)acc[p0]);
            add96(acc[p1], hi[p1], (uint32_t)(acc[p0] >> 32), hi[p0]);
            const uint32_t in = grp_from_above<G>((uint32_t)acc[p0]);
            acc[p0] = in;
            hi[p0] = 0;
        }
    }
    grp_normalise<S, G>(high, acc, hi);
}

}  // namespace rsagpu
