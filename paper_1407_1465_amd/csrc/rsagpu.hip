// Host side of librsagpu.so: argument checks, execution plans, per-device
// state and launches.  No arithmetic happens here.
#include "../../include/rsagpu.h"
#include "registry.hpp"

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>

namespace rsagpu {

// CRT launchers of an instance, null where it is wider than any CRT half.
template <int S, int G, int B>
constexpr crt_launcher crt_of()
{
    if constexpr (crt_instance(S, B)) return &launch_crt<S, G, B>;
    else return nullptr;
}
template <int S, int G, int B>
constexpr ops_launcher ops_crt_of()
{
    if constexpr (crt_instance(S, B)) return &launch_ops_crt<S, G, B>;
    else return nullptr;
}
template <int S, int G, int B>
constexpr ops_launcher ops_crt_pairs_of()
{
    if constexpr (crt_instance(S, B)) return &launch_ops_crt_pairs<S, G, B>;
    else return nullptr;
}

static const Instance kInstances[] = {
#define X(B_, S_, G_)                                                                                     \
    {B_, S_, G_, &launch_modexp<S_, G_, B_>, crt_of<S_, G_, B_>(), &launch_setup<S_, G_, B_>,             \
     &launch_ops_enc<S_, G_, B_>, ops_crt_of<S_, G_, B_>(), ops_crt_pairs_of<S_, G_, B_>(),               \
     &ops_blocks_per_cu<S_, G_, B_>},
#include "instances.def"
#undef X
};

// Width classes in 32-bit limbs; a call runs at the smallest class that holds
// its `limbs`.  kS29 is the limb count of the same class in radix 2^29
// (29 * kS29 >= 32 * class), 0 where no radix-2^29 instance exists.
static const int kClasses[] = {2, 4, 8, 12, 16, 24, 32, 48, 64, 96, 128};
static const int kS29[] = {0, 0, 0, 0, 18, 28, 36, 56, 72, 112, 144};
static const int kNumClasses = sizeof(kClasses) / sizeof(kClasses[0]);
static_assert(standard_s29(18) && standard_s29(28) && standard_s29(36) && standard_s29(56) && standard_s29(72) &&
                  standard_s29(112) && standard_s29(144),
              "kS29 and standard_s29 list the same limb counts");

// Default plan per class: limb radix 2^B, lanes per exponentiation G (limbs
// per lane L = S / G) and window bits w, measured on large batches.  From
// 512-bit operands up the reduced radix 2^29 wins (one v_mad_u64_u32 per
// product, no carry handling, despite ~21% more limb products); below, radix
// 2^32.  kind 0 = plain exponentiation, kind 1 = CRT half.  Two effects pull
// against each other: more limbs per lane amortise the per-step cross-lane
// work (broadcast of m, the limb that moves down) over 2L products and give
// each wave more independent multiplications, while the LDS table (the
// 2^(w-1) odd powers of the sliding window, plus an operand buffer where the
// multiplier is read from LDS: S * (64 / G) words each) and the registers
// limit the waves a CU holds.  For 1024-bit halves L = 18 (G = 2) at one
// wave per SIMD beats L = 9 (G = 4) at two; for full 1024-bit exponents
// L = 18 at two waves per SIMD is best.
struct Plan {
    int B;
    int G;
    int w;
};
//
// Kinds 2 and 3 are the same operations inside rsa_ops_batch, whose buckets
// are usually far smaller than a plain batch and run side by side: there a
// narrower group (more waves per operation) and a smaller LDS footprint (room
// for the other buckets' waves) pay off.  Kind 4 is the CRT half of the
// widest class of a bulk ops batch (rsa_ops_batch with at least
// kBulkOps operations), whose end waits for that bucket's last operations.
// For 4096-bit keys kind 3 takes 16 lanes (S = 80): one operation's chain is
// ~1.6x shorter than on 8 lanes for ~1.2x the lane-instructions, and a
// serving batch ends with its 4096-bit decryptions (p99 50 -> 34 ms against
// 8 lanes at the same request rate).  Kind 4 takes 8 lanes: in a bulk
// batch every CRT bucket runs two wave pairs per workgroup, and 4096-bit
// halves on 8 lanes are half as many waves (274 for the mixed batch's 1092
// operations, in 69 four-wave workgroups), which leaves SIMDs to the other
// buckets (the mixed batch 12.12 -> 10.46-10.62 ms with its other plans at
// their defaults, served requests 7536 -> 8326/s through faster bulk
// bursts; a 5-bit window 10.98 ms).  The plain CRT call
// takes 16 lanes and a 5-bit window for 4096-bit keys too: with two wave
// pairs per workgroup, 256, 1092 and 4368 decryptions took 6.2, 7.1 and
// 17.3 ms against 9.8, 10.9 and 20.4 ms on 8 lanes with a 4-bit window.
// Plain 2048-bit exponentiation takes a 3-bit window: its table then fits
// two waves per SIMD (18.4 KB each; 4 bits take 36.9 KB, one wave), which a
// batch above 16384 messages needs: 32768 full-length exponents took 34.5
// ms against 57.5 ms with 4 bits (16.5 and 17.1 ms at 16384), 32768 e = 65537
// encryptions 0.34 against 0.53 ms (the same at 16384).
static const int kKinds = 5;
static const Plan kDefault[kKinds][kNumClasses] = {
    // classes:  2 .. 12 limbs in radix 2^32; 16 .. 128 limbs in radix 2^29
    {{32, 1, 5}, {32, 1, 5}, {32, 1, 4}, {32, 2, 4}, {29, 2, 4}, {29, 4, 4}, {29, 2, 3}, {29, 8, 4},
     {29, 4, 3}, {29, 16, 4}, {29, 16, 3}},
    {{32, 1, 5}, {32, 1, 5}, {32, 1, 4}, {32, 2, 4}, {29, 2, 4}, {29, 4, 4}, {29, 2, 4}, {29, 8, 4},
     {29, 16, 5}, {29, 16, 4}, {29, 16, 3}},
    {{32, 1, 5}, {32, 1, 5}, {32, 1, 4}, {32, 2, 4}, {29, 2, 4}, {29, 4, 4}, {29, 4, 3}, {29, 8, 4},
     {29, 4, 4}, {29, 8, 4}, {29, 16, 3}},
    {{32, 1, 5}, {32, 1, 5}, {32, 1, 4}, {32, 2, 4}, {32, 4, 5}, {29, 4, 4}, {29, 2, 4}, {29, 8, 5},
     {29, 16, 4}, {29, 16, 4}, {29, 16, 3}},
    {{32, 1, 5}, {32, 1, 5}, {32, 1, 4}, {32, 2, 4}, {32, 4, 5}, {29, 4, 4}, {29, 2, 4}, {29, 8, 5},
     {29, 8, 4}, {29, 16, 4}, {29, 16, 3}},
};

static int pack(const Plan &p) { return p.B << 16 | p.G << 8 | p.w; }
static Plan unpack(int v) { return Plan{v >> 16, (v >> 8) & 0xFF, v & 0xFF}; }

// Current plans; overridable with rsa_set_plan.
static std::atomic<int> g_plan[kKinds][kNumClasses];
static std::once_flag g_plan_once;

static void init_plans()
{
    for (int k = 0; k < kKinds; ++k)
        for (int i = 0; i < kNumClasses; ++i) g_plan[k][i].store(pack(kDefault[k][i]));
}

int num_classes() { return kNumClasses; }
int class_width(int i) { return kClasses[i]; }
int class_s29(int i) { return kS29[i]; }

int class_index(int limbs)
{
    for (int i = 0; i < kNumClasses; ++i)
        if (kClasses[i] >= limbs) return i;
    return -1;
}

const Instance *find_instance(int i, int B, int G)
{
    const int S = B == 32 ? kClasses[i] : (B == 29 ? kS29[i] : 0);
    if (S == 0 || G <= 0) return nullptr;
    // radix 2^29 with more lanes than the class's S divides into: the
    // instance with S rounded up to a multiple of G, where one is compiled
    const int Sw = (B == 29 && S % G) ? (S + G - 1) / G * G : S;
    for (const Instance &in : kInstances)
        if (in.B == B && in.S == Sw && in.G == G) return &in;
    return nullptr;
}

const Instance *any_instance(int i, int B)
{
    const int S = B == 32 ? kClasses[i] : (B == 29 ? kS29[i] : 0);
    if (S == 0) return nullptr;
    for (const Instance &in : kInstances)
        if (in.B == B && in.S == S) return &in;
    return nullptr;
}

static bool crt_kind(int kind) { return kind == 1 || kind == 3 || kind == 4; }

bool resolve(int limbs, int kind, Resolved *r)
{
    std::call_once(g_plan_once, init_plans);
    const int i = class_index(limbs);
    if (i < 0) return false;
    const Plan p = unpack(g_plan[kind][i].load());
    r->inst = find_instance(i, p.B, p.G);
    r->w = p.w;
    return r->inst != nullptr && (!crt_kind(kind) || (r->inst->crt && r->inst->ops_crt));
}

// ---- per-device state: the data-error counter ------------------------------
//
// Word 0 counts per-element data errors (kernels add to it atomically); word
// 1 receives the count rsa_device_errors takes.  Static device memory: each
// device holds its own copy, zero when the code object loads, at an address
// looked up once per device.

static __device__ __align__(256) unsigned long long g_err_words[2];

static const int kMaxDevices = 64;
static unsigned long long *g_errs[kMaxDevices];
static int g_cus[kMaxDevices];
static std::mutex g_dev_mutex;

int device_state(unsigned long long **errs, int *cus)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RSA_EHIP;
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    if (!g_errs[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_err_words)) != hipSuccess || !p) return RSA_EHIP;
        // the non-allocating CRT call's static scratch on this device
        if (order_static_init(dev) != 0) return RSA_EHIP;
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) {
            (void)hipGetLastError();
            n = 1;
        }
        g_cus[dev] = n;
        g_errs[dev] = static_cast<unsigned long long *>(p);
    }
    *errs = g_errs[dev];
    if (cus) *cus = g_cus[dev];
    return RSA_OK;
}

// Moves the error count into word 1 and clears it, in one atomic step.
__global__ void k_take_errors(unsigned long long *w) { w[1] = atomicExch(&w[0], 0ull); }

int status_of(hipError_t e)
{
    if (e == hipSuccess) return RSA_OK;
    if (e == hipErrorOutOfMemory) return RSA_ENOMEM;
    return RSA_EHIP;
}

}  // namespace rsagpu

using namespace rsagpu;

extern "C" int rsa_init(void)
{
    unsigned long long *errs = nullptr;
    return device_state(&errs);
}

extern "C" int rsa_modexp_batch(const uint32_t *base, const uint32_t *exp, const uint32_t *mod, uint32_t *out,
                                size_t count, int limbs, hipStream_t stream)
{
    if (limbs < 1 || limbs > RSA_MAX_LIMBS) return RSA_ELIMBS;
    if (count == 0) return RSA_OK;
    if (!base || !exp || !mod || !out) return RSA_EINVAL;
    Resolved r;
    if (!resolve(limbs, 0, &r)) return RSA_ELIMBS;
    if ((count + 64 / r.inst->G - 1) / (64 / r.inst->G) > 0x7FFFFFFFull) return RSA_EINVAL;
    unsigned long long *errs = nullptr;
    const int st = device_state(&errs);
    if (st != RSA_OK) return st;
    return status_of(r.inst->modexp(base, exp, mod, out, count, limbs, r.w, errs, stream));
}

// Wave pairs per workgroup of a plain CRT launch of `count` messages:
// crt_pairs(G), or two for fewer lanes where the messages need more than one
// and at most two workgroups of one pair per CU (the key-grouped order's
// padding stays within that, see key_order_slots) and the kernel's occupancy
// would let a CU take a second one (one-pair workgroups beyond one per CU
// have been measured to share SIMDs: 8736 1024-bit messages, 273
// workgroups, took 1.12 ms against 0.73 ms in workgroups of two pairs, one
// wave per SIMD).  Where the launch fits one one-pair workgroup per CU, or
// fills every SIMD anyway, one pair measured 1-6% faster.
static const int kMaxCrtW = 8;
static std::atomic<int> g_crt_occ[sizeof(kInstances) / sizeof(kInstances[0])][kMaxCrtW];

static int plain_crt_launch_pairs(const Instance *in, int w, size_t count, int cus)
{
    if (crt_pairs(in->G) > 1) return crt_pairs(in->G);
    const size_t pairs = (count + 64 / in->G - 1) / (64 / in->G);
    if (pairs <= (size_t)cus || pairs > 2 * (size_t)cus || w < 1 || w >= kMaxCrtW ||
        !crt_lds_fits(in->S, in->G, in->B, w, 2))
        return 1;
    std::atomic<int> &cached = g_crt_occ[in - kInstances][w];
    int occ = cached.load(std::memory_order_relaxed);
    if (occ == 0) {
        occ = in->blocks_per_cu(2, w, 1);
        if (occ < 1) occ = -1;                  // unknown: keep one pair
        cached.store(occ, std::memory_order_relaxed);
    }
    return occ > 2 ? 2 : 1;
}

extern "C" int rsa_decrypt_crt_batch(const uint32_t *c, const uint32_t *p, const uint32_t *q, const uint32_t *dp,
                                     const uint32_t *dq, const uint32_t *qinv, uint32_t *out, size_t count,
                                     int limbs, hipStream_t stream)
{
    if (limbs < 2 || limbs > RSA_MAX_LIMBS || (limbs & 1)) return RSA_ELIMBS;
    if (count == 0) return RSA_OK;
    if (!c || !p || !q || !dp || !dq || !qinv || !out) return RSA_EINVAL;
    Resolved r;
    if (!resolve(limbs / 2, 1, &r)) return RSA_ELIMBS;
    const size_t ng = 64 / r.inst->G;
    if ((count + ng - 1) / ng > 0x7FFFFFFFull) return RSA_EINVAL;
    unsigned long long *errs = nullptr;
    int cus = 1;
    const int st = device_state(&errs, &cus);
    if (st != RSA_OK) return st;
    // more than one wave's worth of messages: process them grouped by key
    size_t slots = count;
    const unsigned *order = nullptr;
    if (count > ng) {
        slots = key_order_slots(count, ng, (size_t)cus);
        order = key_order(p, dp, dq, count, limbs / 2, ng, slots, stream);
        if (!order) slots = count;
    }
    return status_of(r.inst->crt(c, p, q, dp, dq, qinv, order, out, slots, limbs / 2, r.w,
                                 plain_crt_launch_pairs(r.inst, r.w, count, cus), errs, stream));
}

static_assert(kStaticOrderMax == RSA_CRT_STATIC_MAX_COUNT, "static scratch size and its public limit agree");

extern "C" int rsa_decrypt_crt_batch_static(const uint32_t *c, const uint32_t *p, const uint32_t *q,
                                            const uint32_t *dp, const uint32_t *dq, const uint32_t *qinv,
                                            uint32_t *out, size_t count, int limbs, hipStream_t stream)
{
    if (limbs < 2 || limbs > RSA_MAX_LIMBS || (limbs & 1)) return RSA_ELIMBS;
    if (count == 0) return RSA_OK;
    if (!c || !p || !q || !dp || !dq || !qinv || !out) return RSA_EINVAL;
    if (count > RSA_CRT_STATIC_MAX_COUNT) return RSA_EINVAL;
    Resolved r;
    if (!resolve(limbs / 2, 1, &r)) return RSA_ELIMBS;
    const size_t ng = 64 / r.inst->G;
    unsigned long long *errs = nullptr;
    int cus = 1;
    const int st = device_state(&errs, &cus);
    if (st != RSA_OK) return st;
    size_t slots = count;
    const unsigned *order = nullptr;
    if (count > ng) {
        const size_t want = key_order_slots(count, ng, (size_t)cus);
        slots = want < kStaticOrderMax ? want : kStaticOrderMax;    // >= count
        if (!(order = key_order_static(p, dp, dq, count, limbs / 2, ng, slots, stream))) return RSA_EHIP;
    }
    return status_of(r.inst->crt(c, p, q, dp, dq, qinv, order, out, slots, limbs / 2, r.w,
                                 plain_crt_launch_pairs(r.inst, r.w, count, cus), errs, stream));
}

extern "C" int rsa_get_plan(int limbs, int kind, rsa_plan *plan)
{
    if (!plan || kind < 0 || kind >= kKinds) return RSA_EINVAL;
    if (limbs < 1 || limbs > RSA_MAX_LIMBS) return RSA_ELIMBS;
    Resolved r;
    if (!resolve(limbs, kind, &r)) return RSA_ELIMBS;
    plan->radix_bits = r.inst->B;
    plan->padded_limbs = r.inst->S;
    plan->lanes_per_op = r.inst->G;
    plan->limbs_per_lane = r.inst->S / r.inst->G;
    plan->window_bits = r.w;
    plan->lds_bytes = (int)lds_bytes_for(r.inst->S, r.inst->G, r.inst->B, r.w);
    return RSA_OK;
}

extern "C" int rsa_set_plan(int limbs, int kind, int radix_bits, int lanes_per_op, int window_bits)
{
    if (kind < 0 || kind >= kKinds) return RSA_EINVAL;
    if (limbs < 1 || limbs > RSA_MAX_LIMBS) return RSA_ELIMBS;
    std::call_once(g_plan_once, init_plans);
    const int i = class_index(limbs);
    if (i < 0) return RSA_ELIMBS;
    if (radix_bits == 0 && lanes_per_op == 0 && window_bits == 0) {   // back to the default
        g_plan[kind][i].store(pack(kDefault[kind][i]));
        return RSA_OK;
    }
    const Instance *in = find_instance(i, radix_bits, lanes_per_op);
    if (!in || (crt_kind(kind) && !(in->crt && in->ops_crt))) return RSA_EINVAL;
    if (window_bits < 2 || window_bits > 7) return RSA_EINVAL;
    if (lds_bytes_for(in->S, in->G, in->B, window_bits) > 64 * 1024) return RSA_EINVAL;
    if (crt_kind(kind) && !crt_lds_fits(in->S, in->G, in->B, window_bits, kind == 3 ? 1 : crt_pairs(in->G)))
        return RSA_EINVAL;
    g_plan[kind][i].store(pack(Plan{radix_bits, lanes_per_op, window_bits}));
    return RSA_OK;
}

extern "C" int rsa_device_errors(hipStream_t stream, uint64_t *n_bad)
{
    if (!n_bad) return RSA_EINVAL;
    unsigned long long *errs = nullptr;
    int st = device_state(&errs);
    if (st != RSA_OK) return st;
    // one caller at a time per process: word 1 is shared
    static std::mutex take_mu;
    std::lock_guard<std::mutex> lock(take_mu);
    hipLaunchKernelGGL(k_take_errors, dim3(1), dim3(1), 0, stream, errs);
    hipError_t e = hipGetLastError();
    unsigned long long v = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&v, errs + 1, sizeof(v), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
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

extern "C" int rsa_version(void) { return 10000 + 100 * 1; }
