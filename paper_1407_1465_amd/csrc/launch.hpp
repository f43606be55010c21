// Typed launchers for the kernel instances (limb radix 2^B, S limbs, G lanes
// per exponentiation).  Each kern_*.hip translation unit instantiates the
// widths it owns; rsagpu.hip dispatches to them.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rsagpu {

typedef hipError_t (*modexp_launcher)(const uint32_t *base, const uint32_t *exp, const uint32_t *mod,
                                      uint32_t *out, size_t count, int limbs, int w,
                                      unsigned long long *errs, hipStream_t stream);
// order: the processing order of the messages, `count` slots each holding a
// message index or kOrderHole (a slot with no message), or nullptr (then
// count is the number of messages, in the given order).  pairs: wave pairs
// per workgroup (1 or 2, at least crt_pairs(G)).
typedef hipError_t (*crt_launcher)(const uint32_t *c, const uint32_t *p, const uint32_t *q, const uint32_t *dp,
                                   const uint32_t *dq, const uint32_t *qinv, const unsigned *order, uint32_t *out,
                                   size_t count, int hl, int w, int pairs, unsigned long long *errs,
                                   hipStream_t stream);

struct KeyDev;
struct ModConsts;
struct OpDesc;

typedef hipError_t (*setup_launcher)(const uint32_t *const *mods, const uint32_t *const *mults, const int *words,
                                     ModConsts *outs, int count, hipStream_t stream);
// Persistent bucket kernel: `blocks` workgroups claim operations until the
// bucket (list, *count) is exhausted; with `urgent` its waves issue ahead of
// other kernels' waves on a shared SIMD (the bucket that ends a batch).
typedef hipError_t (*ops_launcher)(const KeyDev *keys, const OpDesc *ops, const unsigned *list,
                                   const unsigned *count, unsigned *counter, const uint32_t *in_pool,
                                   uint32_t *out_pool, int w, int blocks, int urgent, hipStream_t stream);
// Workgroups resident per CU at window w (occupancy query) of an ops-batch
// kernel (kind 0 encryption, 1 CRT with `pairs` pairs of waves) or of the
// plain CRT kernel (kind 2, one pair per workgroup).
typedef int (*ops_occupancy)(int kind, int w, int pairs);

// Radix-2^29 limb counts of the width classes (29 * S >= 32 * width + 10, so
// R > 2^10 n): the limb count a keyset's Montgomery constants are stored
// with.  An instance with another S (the class's count rounded up to a
// multiple of its lanes per group, for 16 lanes) computes its constants
// itself.
__host__ __device__ constexpr bool standard_s29(int S)
{
    return S == 18 || S == 28 || S == 36 || S == 56 || S == 72 || S == 112 || S == 144;
}

// Instances that also serve CRT halves: the half of the widest modulus
// (128 words) has 64 words, S = 64 limbs in radix 2^32 and at most 80 in
// radix 2^29 (72, or 80 rounded up for 16 lanes).  Wider instances exist for
// full-width exponentiation only and compile no CRT kernels.
__host__ __device__ constexpr bool crt_instance(int S, int B) { return B == 32 ? S <= 64 : S <= 80; }

// Instances whose Montgomery products inside the exponentiation take the
// multiplier from registers (1, 2 or 4 lanes per group: at most one DPP quad
// permute per step; 16 lanes in radix 2^29: one DPP row broadcast per step);
// the others read it from LDS.
__host__ __device__ constexpr bool register_products(int B, int G)
{
    return G == 1 || G == 2 || G == 4 || (G == 16 && B < 32);
}

// Operand buffers of S * (64 / G) words in one 64-lane workgroup's LDS for a
// sliding window of w bits: the 2^(w-1) odd powers, plus the operand buffer
// the LDS-multiplier products stage A through (with register products the
// code before and after the exponentiation borrows the table's space for
// it); at least 4 buffers (Montgomery setup and Garner's staging use up to 3).
__host__ __device__ constexpr int lds_entries(int B, int G, int w)
{
    return ((1 << (w - 1)) + (register_products(B, G) ? 0 : 1)) > 4
               ? ((1 << (w - 1)) + (register_products(B, G) ? 0 : 1))
               : 4;
}

inline size_t lds_bytes_for(int S, int G, int B, int w)
{
    return (size_t)lds_entries(B, G, w) * (size_t)S * (size_t)(64 / G) * 4u;
}

// p/q wave pairs per CRT workgroup where a half has G lanes.  A CU that
// receives a second two-wave workgroup while others have none has been
// measured to run both on the same two SIMDs (a launch of 273 such
// workgroups took 1.57x as long as one of 250), so where the waves hold few
// messages (8 or 16 lanes per half: a batch of them is few workgroups, and
// little LDS keeps several resident) a workgroup carries two pairs, one wave
// per SIMD, and half as many workgroups cover a batch.  This is the least
// the plain CRT kernel (k_crt) takes (rsa_decrypt_crt_batch picks 2 for
// fewer lanes too where a batch needs one to two workgroups of one pair per
// CU).  In rsa_ops_batch every CRT bucket of a bulk call (at least kBulkOps
// operations) takes two pairs where the LDS holds them, whatever its lanes
// (the mixed 32768-operation batch 12.4 -> 10.5 ms with tuned plans); the
// buckets of smaller calls keep one pair: beside other buckets' waves a
// four-wave workgroup waits longer for a CU with room on every SIMD (served
// requests' p99 latency rose from 25 to 31-33 ms with two pairs in every
// bucket of every call).
__host__ __device__ constexpr int crt_pairs(int G) { return G >= 8 ? 2 : 1; }

// A slot of a CRT processing order that holds no message (the padding that
// lets each key's run of messages start a wave).
constexpr unsigned kOrderHole = 0xFFFFFFFFu;

// LDS one workgroup may allocate on gfx950, and the CRT kernels' own LDS
// beyond the waves' regions (the ops kernel's claim word, aligned).
constexpr size_t kMaxGroupLds = 160 * 1024;
constexpr size_t kCrtOwnLds = 16;

// A CRT workgroup of `pairs` pairs of waves (each with its window table and
// buffers) of this plan fits in LDS.
inline bool crt_lds_fits(int S, int G, int B, int w, int pairs)
{
    return 2 * (size_t)pairs * lds_bytes_for(S, G, B, w) + kCrtOwnLds <= kMaxGroupLds;
}


template <int S, int G, int B>
hipError_t launch_modexp(const uint32_t *base, const uint32_t *exp, const uint32_t *mod, uint32_t *out,
                         size_t count, int limbs, int w, unsigned long long *errs, hipStream_t stream);

template <int H, int G, int B>
hipError_t launch_crt(const uint32_t *c, const uint32_t *p, const uint32_t *q, const uint32_t *dp,
                      const uint32_t *dq, const uint32_t *qinv, const unsigned *order, uint32_t *out, size_t count,
                      int hl, int w, int pairs, unsigned long long *errs, hipStream_t stream);

template <int S, int G, int B>
hipError_t launch_setup(const uint32_t *const *mods, const uint32_t *const *mults, const int *words,
                        ModConsts *outs, int count, hipStream_t stream);

template <int S, int G, int B>
hipError_t launch_ops_enc(const KeyDev *keys, const OpDesc *ops, const unsigned *list, const unsigned *count,
                          unsigned *counter, const uint32_t *in_pool, uint32_t *out_pool, int w, int blocks,
                          int urgent, hipStream_t stream);

template <int S, int G, int B>
hipError_t launch_ops_crt(const KeyDev *keys, const OpDesc *ops, const unsigned *list, const unsigned *count,
                          unsigned *counter, const uint32_t *in_pool, uint32_t *out_pool, int w, int blocks,
                          int urgent, hipStream_t stream);

// The ops-batch CRT kernel with two pairs per workgroup (invalid where the
// LDS does not hold them).
template <int S, int G, int B>
hipError_t launch_ops_crt_pairs(const KeyDev *keys, const OpDesc *ops, const unsigned *list, const unsigned *count,
                                unsigned *counter, const uint32_t *in_pool, uint32_t *out_pool, int w, int blocks,
                                int urgent, hipStream_t stream);

// Resident workgroups per CU (see ops_occupancy).
template <int S, int G, int B>
int ops_blocks_per_cu(int kind, int w, int pairs);

}  // namespace rsagpu
