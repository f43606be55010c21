// Resident keys and mixed batches of operations (host side + bucketing).
#include "../../include/rsagpu.h"
#include "keyset_kernels.hpp"
#include "registry.hpp"

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <new>

namespace rsagpu {

static_assert(sizeof(OpDesc) == sizeof(rsa_op), "rsa_op layout");

static const int kMaxBuckets = 32;            // 2 kinds x width classes
static const int kKeySlots = 256;             // key ids per bucket ordered apart (id mod 256)
// workspace header: per bucket its size and claim counter, then per bucket
// and key slot a count that becomes a list cursor
static const size_t kWsHeader = (2 * kMaxBuckets + (size_t)kMaxBuckets * kKeySlots) * sizeof(unsigned);

// ---- bucketing kernels -------------------------------------------------------
//
// Operations go into buckets of one (width class of the key, kind), each
// list ordered by key id (a counting sort over id mod kKeySlots), so that
// a bucket kernel's chunks hold one key's operations.  In a CRT bucket each
// key slot's run starts a wave of its own where the runs, rounded up to
// whole waves, fit the list: the gaps hold kOrderHole, and a wave that would
// have taken the end of one key's run and the start of the next (two
// exponents: the slower per-group schedule) takes the end alone.  Invalid
// operations (kind, key id, or an input/output range outside its pool) are
// counted as data errors and dropped.

__global__ void k_bucket_clear(unsigned *hdr)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 2 * kMaxBuckets + (size_t)kMaxBuckets * kKeySlots) hdr[t] = 0u;
}

// Bucket of an operation, or -1 if it is invalid.
__device__ __forceinline__ int op_bucket(const OpDesc &op, const KeyDev *keys, int nkeys,
                                         unsigned long long in_words, unsigned long long out_words)
{
    if (op.kind > 1u || op.key_id < 0 || op.key_id >= nkeys) return -1;
    const KeyDev &k = keys[op.key_id];
    const unsigned long long wds = (unsigned long long)k.words;
    const bool ok = op.in_off <= in_words && wds <= in_words - op.in_off && op.out_off <= out_words &&
                    wds <= out_words - op.out_off;
    return ok ? k.cls * 2 + (int)op.kind : -1;
}

__global__ void k_bucket_count(const OpDesc *__restrict__ ops, unsigned long long nops,
                               const KeyDev *__restrict__ keys, int nkeys, unsigned long long in_words,
                               unsigned long long out_words, unsigned *slots, unsigned long long *errs)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nops) return;
    const OpDesc op = ops[i];
    const int b = op_bucket(op, keys, nkeys, in_words, out_words);
    if (b < 0) {
        atomicAdd(errs, 1ull);
        return;
    }
    atomicAdd(&slots[b * kKeySlots + (op.key_id % kKeySlots)], 1u);
}

// Per bucket, the length its key slots' runs are rounded up to: the
// operations of one wave of its kernel for a CRT bucket, else 1 (a power of
// two).
struct BucketUnits {
    unsigned u[kMaxBuckets];
};

// One workgroup per bucket: exclusive prefix sum of its key-slot counts, each
// rounded up to the bucket's unit when the rounded runs fit in the list's
// `cap` entries, else as they are (in place: they become the list cursors);
// the bucket's size (holes included); kOrderHole in the gaps.  Each wave
// scans its threads' counts with lane shuffles and every thread adds the
// totals of the waves before its own.  The caller keeps the rounded total
// below 2^32.
__global__ __launch_bounds__(kKeySlots) void k_bucket_scan(unsigned *counts, unsigned *slots, unsigned *lists,
                                                           unsigned long long cap, BucketUnits units)
{
    constexpr int WAVES = kKeySlots / 64;
    __shared__ unsigned wsum[WAVES], wpsum[WAVES];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const unsigned mask = units.u[blockIdx.x] - 1u;
    unsigned *sl = slots + (size_t)blockIdx.x * kKeySlots;
    const unsigned v = sl[t], pv = (v + mask) & ~mask;
    unsigned is = v, ips = pv;                  // inclusive scans within the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned a = __shfl_up(is, o), b = __shfl_up(ips, o);
        if (lane >= o) {
            is += a;
            ips += b;
        }
    }
    if (lane == 63) {
        wsum[wv] = is;
        wpsum[wv] = ips;
    }
    __syncthreads();
    unsigned base = 0u, pbase = 0u, tot = 0u, ptot = 0u;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) {
        const unsigned a = wsum[k], b = wpsum[k];
        if (k < wv) {
            base += a;
            pbase += b;
        }
        tot += a;
        ptot += b;
    }
    const bool pad = (unsigned long long)ptot <= cap;
    const unsigned start = pad ? pbase + ips - pv : base + is - v;
    sl[t] = start;
    if (t == kKeySlots - 1) counts[blockIdx.x] = pad ? ptot : tot;
    if (pad) {
        unsigned *l = lists + (unsigned long long)blockIdx.x * cap + start;
        for (unsigned i = v; i < pv; ++i) l[i] = kOrderHole;
    }
}

__global__ void k_bucket_place(const OpDesc *__restrict__ ops, unsigned long long nops,
                               const KeyDev *__restrict__ keys, int nkeys, unsigned long long in_words,
                               unsigned long long out_words, unsigned *slots, unsigned *lists,
                               unsigned long long cap)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nops) return;
    const OpDesc op = ops[i];
    const int b = op_bucket(op, keys, nkeys, in_words, out_words);
    if (b < 0) return;
    const unsigned at = atomicAdd(&slots[b * kKeySlots + (op.key_id % kKeySlots)], 1u);
    lists[(unsigned long long)b * cap + at] = (unsigned)i;
}

// ---- the keyset ------------------------------------------------------------------

struct KeyHostInfo {
    int cls;
    int hcls;
};

}  // namespace rsagpu

struct rsa_keyset {
    int device;
    int max_keys;
    int nkeys;
    size_t key_words;               // device words reserved per key
    uint32_t *blob;                 // key material and constants
    rsagpu::KeyDev *keys;           // device table
    const uint32_t **stage_mods;    // setup staging (device)
    int *stage_words;
    rsagpu::ModConsts *stage_outs;
    rsagpu::KeyHostInfo *info;      // host copy per key
    unsigned class_mask;            // width classes present
    std::mutex mu;
    // Fork/join of the per-bucket kernels: each caller stream has a fork set
    // of its own (streams created on its first forked call), so calls on
    // different caller streams never queue behind each other's buckets.
    // `forks` (at most kStreams) bounds the streams a call forks onto: a
    // process has HIP's default of 4 hardware queues, and streams beyond
    // them share queues and serialise, so callers x (forks + 1) <= 4 keeps
    // every bucket concurrent.
    static const int kStreams = 3;
    static const int kForkSets = 8;
    struct ForkSet {
        hipStream_t caller;
        int made;                       // streams (and their events) created so far
        hipStream_t streams[kStreams];
        hipEvent_t fork;
        hipEvent_t done[kStreams];
    };
    ForkSet forksets[kForkSets];
    int nforksets;
    int forks = kStreams;
    std::mutex launch_mu;
};

namespace rsagpu {

static size_t s_for(int cls, int B) { return B == 32 ? (size_t)class_width(cls) : (size_t)class_s29(cls); }

// Device words one key of class cls (n of `class_width` words) may need.
static size_t key_words_for(int cls, int hcls)
{
    const size_t W = (size_t)class_width(cls), H = (size_t)class_width(hcls);
    size_t w = 2 * W + 5 * H;                                         // n, e, p, q, dp, dq, qinv
    // one, r2 of n; one, r2, r3 of p and q; qinv * R of p
    for (int B : {32, 29}) w += 2 * s_for(cls, B) + 7 * s_for(hcls, B);
    return w;
}

static bool host_gt(const uint32_t *a, const uint32_t *b, int words)
{
    for (int i = words - 1; i >= 0; --i)
        if (a[i] != b[i]) return a[i] > b[i];
    return false;
}

// n == p * q for p, q of h words and n of 2h words (schoolbook product).
static bool host_is_product(const uint32_t *n, const uint32_t *p, const uint32_t *q, int h)
{
    uint32_t *t = new (std::nothrow) uint32_t[2 * h]();
    if (!t) return false;
    for (int j = 0; j < h; ++j) {
        uint64_t c = 0;
        for (int i = 0; i < h; ++i) {
            const uint64_t v = (uint64_t)p[i] * q[j] + t[i + j] + c;
            t[i + j] = (uint32_t)v;
            c = v >> 32;
        }
        t[j + h] = (uint32_t)c;
    }
    const bool eq = memcmp(t, n, sizeof(uint32_t) * 2 * h) == 0;
    delete[] t;
    return eq;
}

static bool any_nonzero(const uint32_t *x, int words)
{
    for (int i = 0; i < words; ++i)
        if (x[i]) return true;
    return false;
}

}  // namespace rsagpu

using namespace rsagpu;

extern "C" int rsa_keyset_create(rsa_keyset **out, int max_keys)
{
    if (!out || max_keys <= 0 || max_keys > (1 << 20)) return RSA_EINVAL;
    *out = nullptr;
    unsigned long long *errs = nullptr;
    int st = device_state(&errs);
    if (st != RSA_OK) return st;
    rsa_keyset *ks = new (std::nothrow) rsa_keyset();
    if (!ks) return RSA_ENOMEM;
    (void)hipGetDevice(&ks->device);
    ks->max_keys = max_keys;
    const int top = num_classes() - 1;
    ks->key_words = key_words_for(top, class_index(class_width(top) / 2));
    hipError_t e = hipMalloc(&ks->blob, ks->key_words * sizeof(uint32_t) * (size_t)max_keys);
    if (e == hipSuccess) e = hipMalloc(&ks->keys, sizeof(KeyDev) * (size_t)max_keys);
    if (e == hipSuccess) e = hipMalloc(&ks->stage_mods, sizeof(uint32_t *) * 4);
    if (e == hipSuccess) e = hipMalloc(&ks->stage_words, sizeof(int) * 4);
    if (e == hipSuccess) e = hipMalloc(&ks->stage_outs, sizeof(ModConsts) * 4);
    ks->info = new (std::nothrow) KeyHostInfo[max_keys];
    if (e != hipSuccess || !ks->info) {
        rsa_keyset_destroy(ks);
        return e == hipSuccess ? RSA_ENOMEM : status_of(e);
    }
    *out = ks;
    return RSA_OK;
}

extern "C" int rsa_keyset_destroy(rsa_keyset *ks)
{
    if (!ks) return RSA_OK;
    (void)hipDeviceSynchronize();
    if (ks->blob) (void)hipFree(ks->blob);
    if (ks->keys) (void)hipFree(ks->keys);
    if (ks->stage_mods) (void)hipFree(ks->stage_mods);
    if (ks->stage_words) (void)hipFree(ks->stage_words);
    if (ks->stage_outs) (void)hipFree(ks->stage_outs);
    for (int i = 0; i < ks->nforksets; ++i) {
        rsa_keyset::ForkSet &f = ks->forksets[i];
        for (int t = 0; t < f.made; ++t) {
            (void)hipStreamDestroy(f.streams[t]);
            (void)hipEventDestroy(f.done[t]);
        }
        (void)hipEventDestroy(f.fork);
    }
    delete[] ks->info;
    delete ks;
    return RSA_OK;
}

extern "C" int rsa_keyset_add(rsa_keyset *ks, int limbs, const uint32_t *n, const uint32_t *e, const uint32_t *p,
                              const uint32_t *q, const uint32_t *dp, const uint32_t *dq, const uint32_t *qinv,
                              int32_t *key_id)
{
    if (!ks || !n || !e || !p || !q || !dp || !dq || !qinv || !key_id) return RSA_EINVAL;
    if (limbs < 2 || limbs > RSA_MAX_LIMBS || (limbs & 1)) return RSA_ELIMBS;
    const int h = limbs / 2;
    // cheap consistency checks of the key material
    if (!(n[0] & 1u) || !(p[0] & 1u) || !(q[0] & 1u) || !host_gt(p, q, h) || !any_nonzero(e, limbs) ||
        !host_is_product(n, p, q, h) || (h == 1 && q[0] < 3u))
        return RSA_EKEY;
    std::lock_guard<std::mutex> lock(ks->mu);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ks->device) return RSA_EINVAL;
    if (ks->nkeys >= ks->max_keys) return RSA_ENOMEM;
    const int id = ks->nkeys;
    const int cls = class_index(limbs), hcls = class_index(h);
    if (cls < 0 || hcls < 0) return RSA_ELIMBS;

    // layout of this key's words in the blob
    uint32_t *base = ks->blob + (size_t)id * ks->key_words;
    const size_t W = (size_t)class_width(cls), Hw = (size_t)class_width(hcls);
    KeyDev kd;
    memset(&kd, 0, sizeof(kd));
    kd.cls = cls;
    kd.words = limbs;
    kd.hwords = h;
    uint32_t *cur = base;
    auto take = [&](size_t words) { uint32_t *r = cur; cur += words; return r; };
    uint32_t *dn = take(W), *de = take(W), *dpp = take(Hw), *dqq = take(Hw), *ddp = take(Hw), *ddq = take(Hw),
             *dqi = take(Hw);
    kd.n = dn; kd.e = de; kd.p = dpp; kd.q = dqq; kd.dp = ddp; kd.dq = ddq; kd.qinv = dqi;
    for (int slot = 0; slot < 2; ++slot) {
        const int B = slot == 0 ? 32 : 29;
        const size_t sn = s_for(cls, B), sh = s_for(hcls, B);
        kd.cn[slot] = ModConsts{sn ? take(sn) : nullptr, sn ? take(sn) : nullptr, nullptr, nullptr};
        kd.cp[slot] = ModConsts{sh ? take(sh) : nullptr, sh ? take(sh) : nullptr, sh ? take(sh) : nullptr,
                                sh ? take(sh) : nullptr};
        kd.cq[slot] = ModConsts{sh ? take(sh) : nullptr, sh ? take(sh) : nullptr, sh ? take(sh) : nullptr,
                                nullptr};
    }
    if ((size_t)(cur - base) > ks->key_words) return RSA_ELIMBS;

    hipError_t err = hipSuccess;
    auto put = [&](uint32_t *dst, const uint32_t *src, int words) {
        if (err == hipSuccess) err = hipMemcpy(dst, src, sizeof(uint32_t) * words, hipMemcpyHostToDevice);
    };
    put(dn, n, limbs); put(de, e, limbs);
    put(dpp, p, h); put(dqq, q, h); put(ddp, dp, h); put(ddq, dq, h); put(dqi, qinv, h);
    if (err != hipSuccess) return status_of(err);

    // Montgomery constants of n (class cls) and p, q (class hcls), each radix
    for (int slot = 0; slot < 2; ++slot) {
        const int B = slot == 0 ? 32 : 29;
        struct Job { int c; const uint32_t *m; const uint32_t *x; int words; ModConsts out; };
        Job jobs[3] = {{cls, dn, nullptr, limbs, kd.cn[slot]}, {hcls, dpp, dqi, h, kd.cp[slot]},
                       {hcls, dqq, nullptr, h, kd.cq[slot]}};
        for (const Job &j : jobs) {
            if (!j.out.one) continue;
            const Instance *in = any_instance(j.c, B);
            if (!in) continue;
            const uint32_t *mp[2] = {j.m, j.x};                     // modulus, multiplier
            err = hipMemcpy(ks->stage_mods, mp, sizeof(mp), hipMemcpyHostToDevice);
            if (err == hipSuccess) err = hipMemcpy(ks->stage_words, &j.words, sizeof(int), hipMemcpyHostToDevice);
            if (err == hipSuccess) err = hipMemcpy(ks->stage_outs, &j.out, sizeof(ModConsts), hipMemcpyHostToDevice);
            if (err == hipSuccess)
                err = in->setup(ks->stage_mods, ks->stage_mods + 1, ks->stage_words, ks->stage_outs, 1, nullptr);
            if (err == hipSuccess) err = hipStreamSynchronize(nullptr);
            if (err != hipSuccess) return status_of(err);
        }
    }
    err = hipMemcpy(ks->keys + id, &kd, sizeof(kd), hipMemcpyHostToDevice);
    if (err != hipSuccess) return status_of(err);
    ks->info[id] = KeyHostInfo{cls, hcls};
    ks->class_mask |= 1u << cls;
    ks->nkeys = id + 1;
    *key_id = id;
    return RSA_OK;
}

extern "C" size_t rsa_ops_workspace_size(size_t max_ops)
{
    return kWsHeader + (size_t)kMaxBuckets * max_ops * sizeof(unsigned);
}

extern "C" int rsa_ops_batch(rsa_keyset *ks, const rsa_op *ops, size_t nops, const uint32_t *in_pool,
                             size_t in_words, uint32_t *out_pool, size_t out_words, void *workspace,
                             size_t ws_bytes, hipStream_t stream)
{
    if (!ks) return RSA_EINVAL;
    if (nops == 0) return RSA_OK;
    // operation indices and bucket counts are 32-bit on the device
    if (nops > 0xffffffffull) return RSA_EINVAL;
    if (!ops || !in_pool || !out_pool || !workspace || ws_bytes < rsa_ops_workspace_size(nops)) return RSA_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ks->device) return RSA_EINVAL;
    unsigned long long *errs = nullptr;
    int st = device_state(&errs);
    if (st != RSA_OK) return st;
    const size_t cap = (ws_bytes - kWsHeader) / ((size_t)kMaxBuckets * sizeof(unsigned));
    unsigned *hdr = static_cast<unsigned *>(workspace);
    unsigned *counts = hdr, *counters = hdr + kMaxBuckets, *slots = hdr + 2 * kMaxBuckets;
    unsigned *lists = slots + (size_t)kMaxBuckets * kKeySlots;
    int nkeys;
    unsigned mask;
    {
        std::lock_guard<std::mutex> lock(ks->mu);
        nkeys = ks->nkeys;
        mask = ks->class_mask;
    }
    // Bucket order and plans.  The CRT buckets of the widest classes are the
    // longest (their operations are long dependency chains that a bucket's
    // waves cannot shorten), so each of them gets a keyset stream of its own;
    // the remaining buckets (narrower CRT classes, then all encryptions,
    // widest first) follow each other on the caller's stream, beside them,
    // which then waits for the keyset streams.  The widest CRT bucket's
    // waves also raise their issue priority: every call ends with its
    // operations, whose chains are the longest, so on a SIMD shared with other
    // buckets' waves they issue first.
    int order[kMaxBuckets], nb = 0;
    for (int kind = 1; kind >= 0; --kind)
        for (int cls = num_classes() - 1; cls >= 0; --cls)
            if (mask & (1u << cls)) order[nb++] = cls * 2 + kind;
    Resolved plan[kMaxBuckets];
    int pairs[kMaxBuckets];
    BucketUnits units;
    for (int b = 0; b < kMaxBuckets; ++b) units.u[b] = 1u;
    // rounded runs total at most nops + kKeySlots * 63 per bucket: kept 32-bit
    const bool round_runs = nops + (size_t)kKeySlots * 64 <= (size_t)0xFFFFFFFFu;
    for (int t = 0; t < nb; ++t) {
        const int b = order[t], cls = b / 2, kind = b % 2;
        const int width = kind == 0 ? class_width(cls) : class_width(cls) / 2;
        // the ops-batch plans; a bulk batch's widest CRT bucket, which ends it, its own
        const int pkind = (kind == 1 && t == 0 && nops >= kBulkOps) ? 4 : kind + 2;
        if (!resolve(width, pkind, &plan[t])) return RSA_ELIMBS;
        // the CRT buckets of a bulk batch: two pairs of waves per workgroup
        // where the LDS holds them (see crt_pairs)
        const Instance *in = plan[t].inst;
        pairs[t] = kind == 1 && nops >= kBulkOps && crt_lds_fits(in->S, in->G, in->B, plan[t].w, 2) ? 2 : 1;
        if (kind == 1 && round_runs) units.u[b] = (unsigned)(64 / plan[t].inst->G);
    }
    const unsigned op_blocks = (unsigned)((nops + 255) / 256);
    const OpDesc *od = reinterpret_cast<const OpDesc *>(ops);
    hipLaunchKernelGGL(k_bucket_clear, dim3((unsigned)((kWsHeader / sizeof(unsigned) + 255) / 256)), dim3(256), 0,
                       stream, hdr);
    hipLaunchKernelGGL(k_bucket_count, dim3(op_blocks), dim3(256), 0, stream, od, (unsigned long long)nops, ks->keys,
                       nkeys, (unsigned long long)in_words, (unsigned long long)out_words, slots, errs);
    hipLaunchKernelGGL(k_bucket_scan, dim3(kMaxBuckets), dim3(kKeySlots), 0, stream, counts, slots, lists,
                       (unsigned long long)cap, units);
    hipLaunchKernelGGL(k_bucket_place, dim3(op_blocks), dim3(256), 0, stream, od, (unsigned long long)nops,
                       ks->keys, nkeys, (unsigned long long)in_words, (unsigned long long)out_words, slots, lists,
                       (unsigned long long)cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return status_of(e);
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 1;

    // The buckets run concurrently: the widest CRT buckets each on a stream
    // of the caller stream's fork set, forked from `stream` after the
    // bucketing and joined back into it, so small or latency-bound buckets
    // overlap the large ones.
    std::lock_guard<std::mutex> launch_lock(ks->launch_mu);
    rsa_keyset::ForkSet *fs = nullptr;
    int nfork = ks->forks;
    if (nfork > 0) {
        for (int i = 0; i < ks->nforksets; ++i)
            if (ks->forksets[i].caller == stream) fs = &ks->forksets[i];
        // streams and events are made once per caller stream, as many as the
        // forks asked for so far (never while the caller is being captured
        // into a graph: the call forks onto what exists)
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const bool capturing = hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
        (void)hipGetLastError();
        if (!fs && !capturing && ks->nforksets < rsa_keyset::kForkSets) {
            rsa_keyset::ForkSet &f = ks->forksets[ks->nforksets];
            f = rsa_keyset::ForkSet{};
            f.caller = stream;
            if (hipEventCreateWithFlags(&f.fork, hipEventDisableTiming) != hipSuccess) return RSA_EHIP;
            fs = &ks->forksets[ks->nforksets++];
        }
        if (fs && !capturing) {
            for (; fs->made < nfork; ++fs->made) {
                if (hipStreamCreateWithFlags(&fs->streams[fs->made], hipStreamNonBlocking) != hipSuccess)
                    return RSA_EHIP;
                if (hipEventCreateWithFlags(&fs->done[fs->made], hipEventDisableTiming) != hipSuccess) {
                    (void)hipStreamDestroy(fs->streams[fs->made]);
                    return RSA_EHIP;
                }
            }
        }
        nfork = fs ? (nfork < fs->made ? nfork : fs->made) : 0;    // no fork set: every bucket on `stream`
    }
    if (nfork > 0 && (e = hipEventRecord(fs->fork, stream)) != hipSuccess) return status_of(e);
    int forked = 0;
    for (int t = 0; t < nb; ++t) {
        const int b = order[t], kind = b % 2;
        const Resolved &r = plan[t];
        int per = r.inst->blocks_per_cu(kind, r.w, pairs[t]);
        if (per <= 0) per = 1;
        const int blocks = per * cus;
        const bool fork = kind == 1 && t < nfork;
        hipStream_t s = fork ? fs->streams[t] : stream;
        if (fork && (e = hipStreamWaitEvent(s, fs->fork, 0)) != hipSuccess) return status_of(e);
        const ops_launcher fn = kind == 0 ? r.inst->ops_enc : (pairs[t] > 1 ? r.inst->ops_crt_pairs : r.inst->ops_crt);
        e = fn(ks->keys, reinterpret_cast<const OpDesc *>(ops), lists + (size_t)b * cap, counts + b, counters + b,
               in_pool, out_pool, r.w, blocks, (kind == 1 && t == 0) ? 1 : 0, s);
        if (e != hipSuccess) return status_of(e);
        if (fork) {
            if ((e = hipEventRecord(fs->done[t], s)) != hipSuccess) return status_of(e);
            ++forked;
        }
    }
    for (int t = 0; t < forked; ++t)
        if ((e = hipStreamWaitEvent(stream, fs->done[t], 0)) != hipSuccess) return status_of(e);
    return RSA_OK;
}

extern "C" int rsa_keyset_set_forks(rsa_keyset *ks, int forks)
{
    if (!ks || forks < 0 || forks > rsa_keyset::kStreams) return RSA_EINVAL;
    std::lock_guard<std::mutex> launch_lock(ks->launch_mu);
    ks->forks = forks;
    return RSA_OK;
}
