// Definitions of the typed launchers; included by the kern_s<S>.hip units.
#pragma once

#include "launch.hpp"
#include "keyset_kernels.hpp"

namespace rsagpu {

template <int S, int G, int B>
hipError_t launch_modexp(const uint32_t *base, const uint32_t *exp, const uint32_t *mod, uint32_t *out,
                         size_t count, int limbs, int w, unsigned long long *errs, hipStream_t stream)
{
    const size_t ng = 64 / G;
    const size_t blocks = (count + ng - 1) / ng;
    hipLaunchKernelGGL((k_modexp<S, G, B>), dim3((unsigned)blocks), dim3(64), lds_bytes_for(S, G, B, w), stream, base,
                       exp, mod, out, (unsigned long long)count, limbs, w, errs);
    return hipGetLastError();
}

template <int H, int G, int B>
hipError_t launch_crt(const uint32_t *c, const uint32_t *p, const uint32_t *q, const uint32_t *dp,
                      const uint32_t *dq, const uint32_t *qinv, const unsigned *order, uint32_t *out, size_t count,
                      int hl, int w, int pairs, unsigned long long *errs, hipStream_t stream)
{
    const int P = pairs;
    if (P < crt_pairs(G) || P > 2 || !crt_lds_fits(H, G, B, w, P)) return hipErrorInvalidValue;
    const size_t ng = (size_t)(64 / G) * P;    // slots per workgroup (P pairs of waves)
    const size_t blocks = (count + ng - 1) / ng;
    hipLaunchKernelGGL((k_crt<H, G, B>), dim3((unsigned)blocks), dim3(128 * P), 2 * P * lds_bytes_for(H, G, B, w),
                       stream, c, p, q, dp, dq, qinv, order, out, (unsigned long long)count, hl, w, errs);
    return hipGetLastError();
}

template <int S, int G, int B>
hipError_t launch_setup(const uint32_t *const *mods, const uint32_t *const *mults, const int *words,
                        ModConsts *outs, int count, hipStream_t stream)
{
    const int ng = 64 / G;
    const int blocks = (count + ng - 1) / ng;
    hipLaunchKernelGGL((k_setup<S, G, B>), dim3(blocks), dim3(64), lds_bytes_for(S, G, B, 2), stream, mods, mults,
                       words, outs, count);
    return hipGetLastError();
}

template <int S, int G, int B>
hipError_t launch_ops_enc(const KeyDev *keys, const OpDesc *ops, const unsigned *list, const unsigned *count,
                          unsigned *counter, const uint32_t *in_pool, uint32_t *out_pool, int w, int blocks,
                          int urgent, hipStream_t stream)
{
    hipLaunchKernelGGL((k_ops_enc<S, G, B>), dim3(blocks), dim3(64), lds_bytes_for(S, G, B, w), stream, keys, ops,
                       list, count, counter, in_pool, out_pool, w, urgent);
    return hipGetLastError();
}

template <int S, int G, int B>
hipError_t launch_ops_crt(const KeyDev *keys, const OpDesc *ops, const unsigned *list, const unsigned *count,
                          unsigned *counter, const uint32_t *in_pool, uint32_t *out_pool, int w, int blocks,
                          int urgent, hipStream_t stream)
{
    if (!crt_lds_fits(S, G, B, w, 1)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_ops_crt<S, G, B, 1>), dim3(blocks), dim3(128), 2 * lds_bytes_for(S, G, B, w), stream, keys,
                       ops, list, count, counter, in_pool, out_pool, w, urgent);
    return hipGetLastError();
}

template <int S, int G, int B>
hipError_t launch_ops_crt_pairs(const KeyDev *keys, const OpDesc *ops, const unsigned *list, const unsigned *count,
                                unsigned *counter, const uint32_t *in_pool, uint32_t *out_pool, int w, int blocks,
                                int urgent, hipStream_t stream)
{
    if (!crt_lds_fits(S, G, B, w, 2)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_ops_crt<S, G, B, 2>), dim3(blocks), dim3(256), 4 * lds_bytes_for(S, G, B, w), stream, keys,
                       ops, list, count, counter, in_pool, out_pool, w, urgent);
    return hipGetLastError();
}

template <int S, int G, int B>
int ops_blocks_per_cu(int kind, int w, int pairs)
{
    int nb = 0;
    const size_t lds = lds_bytes_for(S, G, B, w);
    hipError_t e = hipErrorInvalidValue;
    if (kind == 0) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_ops_enc<S, G, B>), 64,
                                                         lds);
    } else if constexpr (crt_instance(S, B)) {
        if (kind == 2) {
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_crt<S, G, B>), 128,
                                                             2 * lds);
            return e == hipSuccess ? nb : 0;
        }
        if (pairs > 1)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_ops_crt<S, G, B, 2>),
                                                             256, 4 * lds);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_ops_crt<S, G, B, 1>),
                                                             128, 2 * lds);
    }
    return e == hipSuccess ? nb : 0;
}

}  // namespace rsagpu

// Every launcher of an instance; RSAGPU_INSTANTIATE_EXP leaves out the CRT
// ones (instances wider than any CRT half, see crt_instance).
#define RSAGPU_INSTANTIATE_EXP(B_, S_, G_)                                                                  \
    template hipError_t rsagpu::launch_modexp<S_, G_, B_>(const uint32_t *, const uint32_t *, const uint32_t *, \
                                                      uint32_t *, size_t, int, int, unsigned long long *,   \
                                                      hipStream_t);                                         \
    template hipError_t rsagpu::launch_setup<S_, G_, B_>(const uint32_t *const *, const uint32_t *const *,  \
                                                         const int *, rsagpu::ModConsts *, int,             \
                                                         hipStream_t);                                      \
    template hipError_t rsagpu::launch_ops_enc<S_, G_, B_>(                                                 \
        const rsagpu::KeyDev *, const rsagpu::OpDesc *, const unsigned *, const unsigned *, unsigned *,     \
        const uint32_t *, uint32_t *, int, int, int, hipStream_t);                                          \
    template int rsagpu::ops_blocks_per_cu<S_, G_, B_>(int, int, int);

#define RSAGPU_INSTANTIATE(B_, S_, G_)                                                                      \
    static_assert(rsagpu::crt_instance(S_, B_), "CRT launchers of an instance wider than any CRT half");    \
    RSAGPU_INSTANTIATE_EXP(B_, S_, G_)                                                                      \
    template hipError_t rsagpu::launch_crt<S_, G_, B_>(const uint32_t *, const uint32_t *, const uint32_t *,    \
                                                   const uint32_t *, const uint32_t *, const uint32_t *,    \
                                                   const unsigned *, uint32_t *, size_t, int, int, int,     \
                                                   unsigned long long *, hipStream_t);                      \
    template hipError_t rsagpu::launch_ops_crt<S_, G_, B_>(                                                 \
        const rsagpu::KeyDev *, const rsagpu::OpDesc *, const unsigned *, const unsigned *, unsigned *,     \
        const uint32_t *, uint32_t *, int, int, int, hipStream_t);                                          \
    template hipError_t rsagpu::launch_ops_crt_pairs<S_, G_, B_>(                                           \
        const rsagpu::KeyDev *, const rsagpu::OpDesc *, const unsigned *, const unsigned *, unsigned *,     \
        const uint32_t *, uint32_t *, int, int, int, hipStream_t);
