// Host side of librsagpu.so: argument checks, execution plans and launches.
#include "../../include/rsagpu.h"
#include "modexp_kernels.hpp"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsagpu {

__device__ unsigned long long g_rsa_errors = 0;

// Kernel widths (limbs) with their lanes per exponentiation (G) and window.
struct PlanRow {
    int S;
    int G;
    int w;
};

// One row per supported padded width: limbs per lane L = S / G stays at 6..16
// so that the per-step cross-lane work is amortised over 2L products, and the
// window is the largest whose LDS table (2^w operand buffers of 64*L words)
// keeps several waves resident per CU.
static const PlanRow kPlans[] = {
    {2, 1, 4},   {4, 1, 4},   {8, 1, 4},   {12, 2, 4},  {16, 2, 4},  {24, 4, 4},
    {32, 4, 4},  {48, 4, 3},  {64, 8, 4},  {96, 8, 3},  {128, 16, 4},
};

static const PlanRow *plan_for(int limbs)
{
    for (const PlanRow &p : kPlans)
        if (p.S >= limbs) return &p;
    return nullptr;
}

static size_t lds_bytes(const PlanRow &p)
{
    // operand buffer + table entries 1 .. 2^w - 1, each S * (64 / G) words
    return (size_t)(1u << p.w) * (size_t)p.S * (size_t)(64 / p.G) * 4u;
}

template <int S, int G>
static hipError_t launch_modexp(const uint32_t *base, const uint32_t *exp, const uint32_t *mod, uint32_t *out,
                                size_t count, int limbs, int w, hipStream_t stream)
{
    const size_t ng = 64 / G;
    const size_t blocks = (count + ng - 1) / ng;
    const size_t lds = (size_t)(1u << w) * (size_t)S * ng * 4u;
    hipLaunchKernelGGL((k_modexp<S, G>), dim3((unsigned)blocks), dim3(64), lds, stream, base, exp, mod, out,
                       (unsigned long long)count, limbs, w);
    return hipGetLastError();
}

template <int H, int G>
static hipError_t launch_crt(const uint32_t *c, const uint32_t *p, const uint32_t *q, const uint32_t *dp,
                             const uint32_t *dq, const uint32_t *qinv, uint32_t *out, size_t count, int hl, int w,
                             hipStream_t stream)
{
    const size_t pairs = 64 / G / 2;
    const size_t blocks = (count + pairs - 1) / pairs;
    const size_t lds = (size_t)(1u << w) * (size_t)H * (64 / G) * 4u;
    hipLaunchKernelGGL((k_crt<H, G>), dim3((unsigned)blocks), dim3(64), lds, stream, c, p, q, dp, dq, qinv, out,
                       (unsigned long long)count, hl, w);
    return hipGetLastError();
}

#define RSAGPU_FOR_EACH_PLAN(X) \
    X(2, 1) X(4, 1) X(8, 1) X(12, 2) X(16, 2) X(24, 4) X(32, 4) X(48, 4) X(64, 8) X(96, 8) X(128, 16)

static hipError_t dispatch_modexp(const PlanRow &pl, const uint32_t *base, const uint32_t *exp,
                                  const uint32_t *mod, uint32_t *out, size_t count, int limbs, hipStream_t s)
{
#define X(S_, G_) \
    if (pl.S == S_ && pl.G == G_) return launch_modexp<S_, G_>(base, exp, mod, out, count, limbs, pl.w, s);
    RSAGPU_FOR_EACH_PLAN(X)
#undef X
    return hipErrorInvalidValue;
}

static hipError_t dispatch_crt(const PlanRow &pl, const uint32_t *c, const uint32_t *p, const uint32_t *q,
                               const uint32_t *dp, const uint32_t *dq, const uint32_t *qinv, uint32_t *out,
                               size_t count, int hl, hipStream_t s)
{
#define X(S_, G_) \
    if (pl.S == S_ && pl.G == G_) return launch_crt<S_, G_>(c, p, q, dp, dq, qinv, out, count, hl, pl.w, s);
    RSAGPU_FOR_EACH_PLAN(X)
#undef X
    return hipErrorInvalidValue;
}

static int status_of(hipError_t e)
{
    if (e == hipSuccess) return RSA_OK;
    if (e == hipErrorOutOfMemory) return RSA_ENOMEM;
    return RSA_EHIP;
}

}  // namespace rsagpu

using namespace rsagpu;

extern "C" int rsa_modexp_batch(const uint32_t *base, const uint32_t *exp, const uint32_t *mod, uint32_t *out,
                                size_t count, int limbs, hipStream_t stream)
{
    if (limbs < 1 || limbs > RSA_MAX_LIMBS) return RSA_ELIMBS;
    if (count == 0) return RSA_OK;
    if (!base || !exp || !mod || !out) return RSA_EINVAL;
    const PlanRow *pl = plan_for(limbs);
    if (!pl) return RSA_ELIMBS;
    if ((count + 64 / pl->G - 1) / (64 / pl->G) > 0x7FFFFFFFull) return RSA_EINVAL;
    return status_of(dispatch_modexp(*pl, base, exp, mod, out, count, limbs, stream));
}

extern "C" int rsa_decrypt_crt_batch(const uint32_t *c, const uint32_t *p, const uint32_t *q, const uint32_t *dp,
                                     const uint32_t *dq, const uint32_t *qinv, uint32_t *out, size_t count,
                                     int limbs, hipStream_t stream)
{
    if (limbs < 2 || limbs > RSA_MAX_LIMBS || (limbs & 1)) return RSA_ELIMBS;
    if (count == 0) return RSA_OK;
    if (!c || !p || !q || !dp || !dq || !qinv || !out) return RSA_EINVAL;
    const PlanRow *pl = plan_for(limbs / 2);
    if (!pl) return RSA_ELIMBS;
    if (pl->G > 32) return RSA_ELIMBS;
    if ((count + 32 / pl->G - 1) / (32 / pl->G) > 0x7FFFFFFFull) return RSA_EINVAL;
    return status_of(dispatch_crt(*pl, c, p, q, dp, dq, qinv, out, count, limbs / 2, stream));
}

extern "C" int rsa_get_plan(int limbs, int kind, rsa_plan *plan)
{
    if (!plan || (kind != 0 && kind != 1)) return RSA_EINVAL;
    if (limbs < 1 || limbs > RSA_MAX_LIMBS) return RSA_ELIMBS;
    const PlanRow *pl = plan_for(limbs);
    if (!pl) return RSA_ELIMBS;
    plan->padded_limbs = pl->S;
    plan->lanes_per_op = pl->G;
    plan->limbs_per_lane = pl->S / pl->G;
    plan->window_bits = pl->w;
    plan->lds_bytes = (int)lds_bytes(*pl);
    return RSA_OK;
}

extern "C" int rsa_device_errors(hipStream_t stream, uint64_t *n_bad)
{
    if (!n_bad) return RSA_EINVAL;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return status_of(e);
    unsigned long long v = 0, zero = 0;
    e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_rsa_errors), sizeof(v), 0, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return status_of(e);
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_rsa_errors), &zero, sizeof(zero), 0, hipMemcpyHostToDevice);
    if (e != hipSuccess) return status_of(e);
    *n_bad = v;
    return RSA_OK;
}

extern "C" const char *rsa_status_str(int status)
{
    switch (status) {
    case RSA_OK: return "ok";
    case RSA_EINVAL: return "invalid argument";
    case RSA_ELIMBS: return "limb width out of range";
    case RSA_ENOMEM: return "out of device memory";
    case RSA_EHIP: return "HIP runtime error";
    case RSA_EKEY: return "malformed key";
    default: return "unknown status";
    }
}

extern "C" int rsa_version(void) { return 100; }
