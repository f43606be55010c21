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
typedef hipError_t (*crt_launcher)(const uint32_t *c, const uint32_t *p, const uint32_t *q, const uint32_t *dp,
                                   const uint32_t *dq, const uint32_t *qinv, uint32_t *out, size_t count, int hl,
                                   int w, unsigned long long *errs, hipStream_t stream);

// LDS bytes of one 64-lane workgroup: 2^w operand buffers of S * (64 / G) words.
inline size_t lds_bytes_for(int S, int G, int w) { return (size_t)(1u << w) * (size_t)S * (size_t)(64 / G) * 4u; }

template <int S, int G, int B>
hipError_t launch_modexp(const uint32_t *base, const uint32_t *exp, const uint32_t *mod, uint32_t *out,
                         size_t count, int limbs, int w, unsigned long long *errs, hipStream_t stream);

template <int H, int G, int B>
hipError_t launch_crt(const uint32_t *c, const uint32_t *p, const uint32_t *q, const uint32_t *dp,
                      const uint32_t *dq, const uint32_t *qinv, uint32_t *out, size_t count, int hl, int w,
                      unsigned long long *errs, hipStream_t stream);

}  // namespace rsagpu
