// Issue-rate probe of the VALU's 32-bit integer multiplies on gfx950 (the
// instructions every Montgomery product of the RSA kernels is made of).
// Each lane runs MULPEAK_CHAINS independent dependency chains, so with
// several waves per SIMD the rate measured is the issue rate of the
// instruction, not its latency.
#include "../../include/mulpeak.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

template <int OP>
__global__ __launch_bounds__(MULPEAK_LANES) void k_mulpeak(const uint32_t *__restrict__ seed,
                                                           uint64_t *__restrict__ sink, int iters)
{
    const unsigned t = blockIdx.x * MULPEAK_LANES + threadIdx.x;
    const uint32_t y = seed[t % MULPEAK_SEED_WORDS] | 1u;
    uint64_t acc[MULPEAK_CHAINS];
    uint32_t x[MULPEAK_CHAINS];
#pragma unroll
    for (int k = 0; k < MULPEAK_CHAINS; ++k) {
        const uint32_t s = seed[(t + 7u * k + 1u) % MULPEAK_SEED_WORDS];
        acc[k] = ((uint64_t)s << 32) | (s ^ 0x9E3779B9u);
        x[k] = s | 1u;
    }
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < MULPEAK_CHAINS; ++k) {
            if constexpr (OP == 0) acc[k] = (uint64_t)(uint32_t)acc[k] * y + acc[k];
            else if constexpr (OP == 1) x[k] = x[k] * x[k];   // squaring: no two steps fold into one
            else x[k] = __umulhi(x[k], y);
        }
    }
    uint64_t fold = 0;
#pragma unroll
    for (int k = 0; k < MULPEAK_CHAINS; ++k) fold ^= OP == 0 ? acc[k] : (uint64_t)x[k] << (k & 31);
    sink[t] = fold;
}

}  // namespace

extern "C" int mulpeak_launch(int op, const uint32_t *seed, uint64_t *sink, int blocks, int iters,
                              hipStream_t stream)
{
    if (!seed || !sink || op < 0 || op > 2 || blocks < 1 || iters < 1) return -1;
    const dim3 grid((unsigned)blocks), block(MULPEAK_LANES);
    if (op == 0) hipLaunchKernelGGL(k_mulpeak<0>, grid, block, 0, stream, seed, sink, iters);
    else if (op == 1) hipLaunchKernelGGL(k_mulpeak<1>, grid, block, 0, stream, seed, sink, iters);
    else hipLaunchKernelGGL(k_mulpeak<2>, grid, block, 0, stream, seed, sink, iters);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}
