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
// CRT material is made smaller than "p" by clearing its top bit.  The values
// are not RSA keys - only their shape matters for timing.
__global__ void k_fill(uint32_t *p, unsigned long long nwords, int words_per_item, unsigned long long salt,
                       int mode)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nwords) return;
    unsigned long long z = (i + 1) * 0x9E3779B97F4A7C15ull + salt;
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

static hipError_t fill(uint32_t *p, size_t items, int words, unsigned long long salt, int mode, hipStream_t s)
{
    const unsigned long long n = (unsigned long long)items * (unsigned long long)words;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, words, salt, mode);
    return hipGetLastError();
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

}  // namespace rsagpu

using namespace rsagpu;

extern "C" int rsa_autotune(int limbs, int kind, int exp_bits, size_t count, hipStream_t stream, rsa_plan *best)
{
    if (kind != 0 && kind != 1) return RSA_EINVAL;
    if (limbs < 1 || limbs > RSA_MAX_LIMBS || (kind == 1 && ((limbs & 1) || limbs < 2))) return RSA_ELIMBS;
    if (count == 0 || count > (1u << 22)) return RSA_EINVAL;
    const int width = kind == 0 ? limbs : limbs / 2;          // plan class width
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
    auto release = [&]() {
        (void)hipStreamSynchronize(stream);
        for (void *p : bufs) (void)hipFree(p);
        bufs.clear();
    };
    const int h = limbs / 2;
    uint32_t *a = nullptr, *b = nullptr, *m = nullptr, *out = nullptr, *p = nullptr, *q = nullptr, *dp = nullptr,
             *dq = nullptr, *qi = nullptr;
    hipError_t e = hipSuccess;
    if (kind == 0) {
        a = alloc(count * limbs); b = alloc(count * limbs); m = alloc(count * limbs); out = alloc(count * limbs);
        if (!a || !b || !m || !out) { release(); return RSA_ENOMEM; }
        e = fill(m, count, limbs, 1, 1, stream);
        if (e == hipSuccess) e = fill(a, count, limbs, 2, 3, stream);
        if (e == hipSuccess) e = fill(b, count, limbs, 3, 0, stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_exp_mask, dim3((unsigned)((count * limbs + 255) / 256)), dim3(256), 0, stream, b,
                               (unsigned long long)count, limbs, exp_bits);
            e = hipGetLastError();
        }
    } else {
        a = alloc(count * limbs); out = alloc(count * limbs);
        p = alloc(count * h); q = alloc(count * h); dp = alloc(count * h); dq = alloc(count * h);
        qi = alloc(count * h);
        if (!a || !out || !p || !q || !dp || !dq || !qi) { release(); return RSA_ENOMEM; }
        e = fill(p, count, h, 4, 1, stream);
        if (e == hipSuccess) e = fill(q, count, h, 5, 2, stream);
        if (e == hipSuccess) e = fill(a, count, limbs, 6, 3, stream);
        if (e == hipSuccess) e = fill(dp, count, h, 7, 0, stream);
        if (e == hipSuccess) e = fill(dq, count, h, 8, 0, stream);
        if (e == hipSuccess) e = fill(qi, count, h, 9, 2, stream);
        for (uint32_t *x : {dp, dq}) {
            if (e != hipSuccess) break;
            hipLaunchKernelGGL(k_exp_mask, dim3((unsigned)((count * h + 255) / 256)), dim3(256), 0, stream, x,
                               (unsigned long long)count, h, exp_bits);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) { release(); return status_of(e); }

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { release(); return RSA_EHIP; }
    float best_ms = -1.0f;
    int bB = 0, bG = 0, bw = 0;
    for (int B : {32, 29}) {
        for (int G : {1, 2, 4, 8, 16}) {
            if (!find_instance(cls, B, G)) continue;
            if (kind == 1 && 64 / G < 2) continue;
            for (int w = 2; w <= 6; ++w) {
                if (rsa_set_plan(width, kind, B, G, w) != RSA_OK) continue;
                auto run = [&]() {
                    return kind == 0 ? rsa_modexp_batch(a, b, m, out, count, limbs, stream)
                                     : rsa_decrypt_crt_batch(a, p, q, dp, dq, qi, out, count, limbs, stream);
                };
                if (run() != RSA_OK) continue;                         // warm-up
                (void)hipEventRecord(e0, stream);
                int okruns = 0;
                for (int r = 0; r < 3; ++r) okruns += run() == RSA_OK;
                (void)hipEventRecord(e1, stream);
                if (hipEventSynchronize(e1) != hipSuccess || okruns != 3) continue;
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (best_ms < 0.0f || ms < best_ms) { best_ms = ms; bB = B; bG = G; bw = w; }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    release();
    if (best_ms < 0.0f) {
        (void)rsa_set_plan(width, kind, 0, 0, 0);
        return RSA_EHIP;
    }
    st = rsa_set_plan(width, kind, bB, bG, bw);
    if (st == RSA_OK && best) st = rsa_get_plan(width, kind, best);
    return st;
}
