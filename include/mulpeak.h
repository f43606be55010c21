/*
 * mulpeak.h - C ABI of libmulpeak.so, the issue-rate probe for the 32-bit
 * integer multiplies that bound the modular-exponentiation kernels of
 * librsagpu.so (a Montgomery product of s limbs is 2s^2 + s 32x32-bit
 * products; the paper's Section 3.6 makes exponentiation a chain of such
 * products).  It is a measurement tool, not part of the RSA path: it gives
 * the multiply rate the chip sustains, which the roofline of the RSA kernels
 * is quoted against beside the nominal rate (one product per lane per clock).
 *
 * A launch runs `blocks` workgroups of MULPEAK_LANES lanes; every lane runs
 * MULPEAK_CHAINS independent chains of `iters` operations each, so the
 * measured time is issue throughput, not latency:
 *   op 0: v_mad_u64_u32  (x = lo32(x) * y + x, 64-bit x)
 *   op 1: v_mul_lo_u32   (x = x * x mod 2^32; a chain x * y * y ... would
 *                         let the compiler fold steps into one product)
 *   op 2: v_mul_hi_u32   (x = (x * y) >> 32)
 * Operations per launch = blocks * MULPEAK_LANES * MULPEAK_CHAINS * iters.
 *
 * seed: MULPEAK_SEED_WORDS device words (any values); sink: blocks *
 * MULPEAK_LANES device 64-bit words, each lane's chains folded together (so
 * no chain is dead code).  Both are caller-owned device memory; the launch
 * is asynchronous on `stream`.  Returns 0, -1 for an invalid argument (null
 * pointer, op outside 0..2, blocks or iters < 1), -4 if the launch failed.
 */
#ifndef MULPEAK_H
#define MULPEAK_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MULPEAK_LANES 256
#define MULPEAK_CHAINS 16
#define MULPEAK_SEED_WORDS 256

int mulpeak_launch(int op, const uint32_t *seed, uint64_t *sink, int blocks, int iters, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* MULPEAK_H */
