// Plan autotuner: times every compiled kernel instance of a width class at
// every window that fits, on synthetic operands of the caller's batch size,
// and installs the fastest plan.
#include "../../include/rsagpu.h"
#include "registry.hpp"

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace rsagpu {

// Fills synthetic operands: every word pseudo-random (SplitMix64 of the word
// index and a salt); moduli get their top bit and bit 0 set, the "q" half of
// CRT material is made smaller than "p" by clearing its top bit.  With
// period > 0 item i repeats item i mod period (operands shared by the
// elements of one key, as in the workloads: one exponent per key, so waves
// run the shared-exponent schedule).  The values are not RSA keys - only
// their shape matters for timing.
__global__ void k_fill(uint32_t *p, unsigned long long nwords, int words_per_item, unsigned long long salt,
                       int mode, unsigned long long period)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nwords) return;
    const unsigned long long wpi = (unsigned long long)words_per_item;
    const unsigned long long src = period ? (i / wpi) % period * wpi + i % wpi : i;
    unsigned long long z = (src + 1) * 0x9E3779B97F4A7C15ull + salt;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    uint32_t v = (uint32_t)z;
    const int k = (int)(i % (unsigned long long)words_per_item);
    if (mode == 1) {                                   // odd modulus, top bit set
        if (k == 0) v |= 1u;
        if (k == words_per_item - 1) v |= 0x80000000u;
    } else if (mode == 2) {                            // odd, smaller than any mode-1 value
        if (k == 0) v |= 1u;
        if (k == words_per_item - 1) v &= 0x7FFFFFFFu;
    } else if (mode == 3) {                            // below a mode-1 modulus
        if (k == words_per_item - 1) v &= 0x3FFFFFFFu;
    }
    p[i] = v;
}

static hipError_t fill(uint32_t *p, size_t items, int words, unsigned long long salt, int mode, hipStream_t s,
                       unsigned long long period = 0)
{
    const unsigned long long n = (unsigned long long)items * (unsigned long long)words;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, words, salt, mode,
                       period);
    return hipGetLastError();
}

// Host SplitMix64 (the same generator as k_fill, for synthetic key material).
static uint64_t splitmix64(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Exponent of exp_bits bits (top bit set, rest random) in every item.
__global__ void k_exp_mask(uint32_t *p, unsigned long long items, int words, int exp_bits)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= items * (unsigned long long)words) return;
    const int k = (int)(i % (unsigned long long)words);
    const int top = exp_bits - 1;
    uint32_t v = p[i];
    if (32 * k > top) v = 0;
    else if (32 * k + 31 >= top) {
        const int b = top - 32 * k;
        v = (v & ((b == 31) ? 0xFFFFFFFFu : ((1u << (b + 1)) - 1u))) | (1u << b);
    }
    p[i] = v;
}

// Synthetic key material for a keyset of width `limbs` (h = limbs / 2 words
// per prime): p and q with their top two bits set and p > q, both odd,
// n = p * q (so every input below 2^(32 limbs - 2) is below n), e = 65537,
// full-length dp and dq, qinv below p.  Not RSA keys: timing only.
struct SynthKey {
    std::vector<uint32_t> n, e, p, q, dp, dq, qinv;
};

static SynthKey synth_key(int limbs, uint64_t seed)
{
    const int h = limbs / 2;
    SynthKey k;
    k.n.assign(limbs, 0); k.e.assign(limbs, 0);
    k.p.resize(h); k.q.resize(h); k.dp.resize(h); k.dq.resize(h); k.qinv.resize(h);
    for (int i = 0; i < h; ++i) {
        k.p[i] = (uint32_t)splitmix64(seed);
        k.q[i] = (uint32_t)splitmix64(seed);
        k.dp[i] = (uint32_t)splitmix64(seed);
        k.dq[i] = (uint32_t)splitmix64(seed);
        k.qinv[i] = (uint32_t)splitmix64(seed);
    }
    k.p[0] |= 1u; k.q[0] |= 1u;
    k.p[h - 1] = 0xF0000000u | (k.p[h - 1] & 0x0FFFFFFFu);
    k.q[h - 1] = 0xC0000000u | (k.q[h - 1] & 0x0FFFFFFFu);
    k.dp[h - 1] |= 0x80000000u; k.dq[h - 1] |= 0x80000000u;
    k.qinv[h - 1] &= 0x7FFFFFFFu;
    for (int j = 0; j < h; ++j) {                   // n = p * q, schoolbook
        uint64_t c = 0;
        for (int i = 0; i < h; ++i) {
            const uint64_t v = (uint64_t)k.p[i] * k.q[j] + k.n[i + j] + c;
            k.n[i + j] = (uint32_t)v;
            c = v >> 32;
        }
        k.n[j + h] = (uint32_t)c;
    }
    k.e[0] = 65537u;
    return k;
}

// Timing harness of one kind: runs the call once (warm-up), then three
// times between events; the mean ms, or a negative value if a run failed.
template <typename Run>
static float time_runs(Run run, hipEvent_t e0, hipEvent_t e1, hipStream_t stream)
{
    if (run() != RSA_OK) return -1.0f;
    (void)hipEventRecord(e0, stream);
    int ok = 0;
    for (int r = 0; r < 3; ++r) ok += run() == RSA_OK;
    (void)hipEventRecord(e1, stream);
    if (hipEventSynchronize(e1) != hipSuccess || ok != 3) return -1.0f;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms / 3.0f;
}

}  // namespace rsagpu

using namespace rsagpu;

extern "C" int rsa_autotune(int limbs, int kind, int exp_bits, size_t count, hipStream_t stream, rsa_plan *best)
{
    if (kind < 0 || kind > 4) return RSA_EINVAL;
    const bool crt = kind == 1 || kind == 3 || kind == 4;
    if (limbs < 1 || limbs > RSA_MAX_LIMBS || (crt && ((limbs & 1) || limbs < 2))) return RSA_ELIMBS;
    if (kind >= 2 && ((limbs & 1) || limbs < 2)) return RSA_ELIMBS;     // keyset keys have even widths
    if (count == 0 || count > (1u << 22) || (kind >= 2 && count > (1u << 20))) return RSA_EINVAL;
    const int width = crt ? limbs / 2 : limbs;                  // plan class width
    const int ebits_max = 32 * width;
    if (exp_bits <= 0 || exp_bits > ebits_max) exp_bits = ebits_max;
    const int cls = class_index(width);
    if (cls < 0) return RSA_ELIMBS;
    unsigned long long *errs = nullptr;
    int st = device_state(&errs);
    if (st != RSA_OK) return st;

    // synthetic operands (freed before returning)
    std::vector<void *> bufs;
    auto alloc = [&](size_t words) -> uint32_t * {
        void *p = nullptr;
        if (hipMalloc(&p, words * sizeof(uint32_t)) != hipSuccess) return nullptr;
        bufs.push_back(p);
        return static_cast<uint32_t *>(p);
    };
    rsa_keyset *ks = nullptr;
    auto release = [&]() {
        (void)hipStreamSynchronize(stream);
        for (void *p : bufs) (void)hipFree(p);
        bufs.clear();
        if (ks) (void)rsa_keyset_destroy(ks);
        ks = nullptr;
    };
    // kinds 0 and 1 time the plain calls on operands shared per key, as the
    // workloads have them: one modulus and exponent for every element of a
    // plain exponentiation (one key's messages), kKeys keys round-robin for
    // CRT (the call groups each key's messages into waves); kinds 2 to 4
    // time rsa_ops_batch on a keyset of kKeys synthetic keys of this width,
    // operations round-robin over the keys
    const unsigned long long kKeys = 16;
    const int h = limbs / 2;
    uint32_t *a = nullptr, *b = nullptr, *m = nullptr, *out = nullptr, *p = nullptr, *q = nullptr, *dp = nullptr,
             *dq = nullptr, *qi = nullptr;
    void *ops = nullptr, *ws = nullptr;
    size_t ws_bytes = 0;
    hipError_t e = hipSuccess;
    if (kind == 0) {
        a = alloc(count * limbs); b = alloc(count * limbs); m = alloc(count * limbs); out = alloc(count * limbs);
        if (!a || !b || !m || !out) { release(); return RSA_ENOMEM; }
        e = fill(m, count, limbs, 1, 1, stream, 1);
        if (e == hipSuccess) e = fill(a, count, limbs, 2, 3, stream);
        if (e == hipSuccess) e = fill(b, count, limbs, 3, 0, stream, 1);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_exp_mask, dim3((unsigned)((count * limbs + 255) / 256)), dim3(256), 0, stream, b,
                               (unsigned long long)count, limbs, exp_bits);
            e = hipGetLastError();
        }
    } else if (kind == 1) {
        a = alloc(count * limbs); out = alloc(count * limbs);
        p = alloc(count * h); q = alloc(count * h); dp = alloc(count * h); dq = alloc(count * h);
        qi = alloc(count * h);
        if (!a || !out || !p || !q || !dp || !dq || !qi) { release(); return RSA_ENOMEM; }
        e = fill(p, count, h, 4, 1, stream, kKeys);
        if (e == hipSuccess) e = fill(q, count, h, 5, 2, stream, kKeys);
        if (e == hipSuccess) e = fill(a, count, limbs, 6, 3, stream);
        if (e == hipSuccess) e = fill(dp, count, h, 7, 0, stream, kKeys);
        if (e == hipSuccess) e = fill(dq, count, h, 8, 0, stream, kKeys);
        if (e == hipSuccess) e = fill(qi, count, h, 9, 2, stream, kKeys);
        for (uint32_t *x : {dp, dq}) {
            if (e != hipSuccess) break;
            hipLaunchKernelGGL(k_exp_mask, dim3((unsigned)((count * h + 255) / 256)), dim3(256), 0, stream, x,
                               (unsigned long long)count, h, exp_bits);
            e = hipGetLastError();
        }
    } else {
        if ((st = rsa_keyset_create(&ks, (int)kKeys)) != RSA_OK) { release(); return st; }
        for (unsigned long long j = 0; j < kKeys; ++j) {
            const SynthKey k = synth_key(limbs, 0x5EEDull * (j + 1) + (uint64_t)limbs);
            int32_t id = -1;
            st = rsa_keyset_add(ks, limbs, k.n.data(), k.e.data(), k.p.data(), k.q.data(), k.dp.data(),
                                k.dq.data(), k.qinv.data(), &id);
            if (st != RSA_OK) { release(); return st; }
        }
        a = alloc(count * limbs); out = alloc(count * limbs);
        std::vector<rsa_op> host_ops(count);
        for (size_t i = 0; i < count; ++i)
            host_ops[i] = rsa_op{kind == 2 ? 0u : 1u, (int32_t)(i % kKeys), (uint64_t)i * limbs, (uint64_t)i * limbs};
        ws_bytes = rsa_ops_workspace_size(count);
        if (!a || !out || hipMalloc(&ops, sizeof(rsa_op) * count) != hipSuccess) { release(); return RSA_ENOMEM; }
        bufs.push_back(ops);
        if (hipMalloc(&ws, ws_bytes) != hipSuccess) { release(); return RSA_ENOMEM; }
        bufs.push_back(ws);
        e = hipMemcpy(ops, host_ops.data(), sizeof(rsa_op) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = fill(a, count, limbs, 6, 3, stream);
    }
    if (e != hipSuccess) { release(); return status_of(e); }

    // a CRT bucket takes plan kind 3 or 4 by the batch's size and rank, so
    // both are set to the candidate while a CRT kind is timed
    const int twin = kind == 3 ? 4 : (kind == 4 ? 3 : -1);
    rsa_plan twin_saved{};
    if (twin >= 0 && (st = rsa_get_plan(width, twin, &twin_saved)) != RSA_OK) { release(); return st; }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { release(); return RSA_EHIP; }
    float best_ms = -1.0f;
    int bB = 0, bG = 0, bw = 0;
    for (int B : {32, 29}) {
        for (int G : {1, 2, 4, 8, 16}) {
            if (!find_instance(cls, B, G)) continue;
            if (crt && 64 / G < 2) continue;
            for (int w = 2; w <= 6; ++w) {
                if (rsa_set_plan(width, kind, B, G, w) != RSA_OK) continue;
                if (twin >= 0 && rsa_set_plan(width, twin, B, G, w) != RSA_OK) continue;
                auto run = [&]() {
                    if (kind == 0) return rsa_modexp_batch(a, b, m, out, count, limbs, stream);
                    if (kind == 1) return rsa_decrypt_crt_batch(a, p, q, dp, dq, qi, out, count, limbs, stream);
                    return rsa_ops_batch(ks, static_cast<const rsa_op *>(ops), count, a, count * limbs, out,
                                         count * limbs, ws, ws_bytes, stream);
                };
                const float ms = time_runs(run, e0, e1, stream);
                if (ms < 0.0f) continue;
                if (best_ms < 0.0f || ms < best_ms) { best_ms = ms; bB = B; bG = G; bw = w; }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    release();
    if (twin >= 0)
        (void)rsa_set_plan(width, twin, twin_saved.radix_bits, twin_saved.lanes_per_op, twin_saved.window_bits);
    if (best_ms < 0.0f) {
        (void)rsa_set_plan(width, kind, 0, 0, 0);
        return RSA_EHIP;
    }
    st = rsa_set_plan(width, kind, bB, bG, bw);
    if (st == RSA_OK && best) st = rsa_get_plan(width, kind, best);
    return st;
}
