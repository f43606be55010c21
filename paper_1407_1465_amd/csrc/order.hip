// Grouping of a plain CRT batch by key: a processing order in which messages
// under the same key follow each other, so that the waves of the CRT kernel
// mostly hold one key's halves (one exponent per wave: one schedule, symmetric
// squarings).  A counting sort of the messages by a hash of their key words
// (p, dp, dq) into kBuckets = 2^16 buckets; distinct keys that share a
// bucket only share waves, which then take the per-group schedule.  The
// order has `slots` >= count entries, free ones holding kOrderHole.  When
// the buckets' runs, each rounded up to a whole number of waves (ng
// messages), fit in the slots, every run starts a wave of its own: a key
// whose message count is not a multiple of ng then leaves a partly empty
// wave rather than one shared with the next key, which would take the
// slower per-group schedule and hold the whole launch back.  Otherwise the
// runs follow each other with no gaps.  The order changes which messages
// share a wave, never a result.
#include "registry.hpp"

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

namespace rsagpu {

static const int kBucketBits = 16;
static const int kBuckets = 1 << kBucketBits;

__device__ __forceinline__ uint32_t key_bucket(const uint32_t *p, const uint32_t *dp, const uint32_t *dq, size_t i,
                                               int hl)
{
    const size_t o = i * (size_t)hl;
    const uint32_t p1 = hl > 1 ? p[o + 1] : 0u;
    uint32_t h = p[o] * 0x9E3779B1u;
    h ^= (p1 + 0x7F4A7C15u) * 0x85EBCA77u;
    h = (h << 13 | h >> 19) ^ dp[o] * 0xC2B2AE3Du;
    h = (h << 11 | h >> 21) ^ dq[o] * 0x27D4EB2Fu;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return h >> (32 - kBucketBits);
}

__global__ void k_order_clear(unsigned *cnt, unsigned *order, unsigned long long slots)
{
    // fill kernels, not memsets: safe to capture in a graph
    const unsigned long long t = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (unsigned long long)kBuckets) cnt[t] = 0u;
    if (t < slots) order[t] = kOrderHole;
}

__global__ void k_order_count(const uint32_t *p, const uint32_t *dp, const uint32_t *dq, unsigned long long count,
                              int hl, unsigned *cnt)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    atomicAdd(&cnt[key_bucket(p, dp, dq, i, hl)], 1u);
}

// Start of every bucket's run: the exclusive prefix sum of the bucket
// counts, each rounded up to a multiple of ng (a power of two; 1 rounds
// nothing) when the rounded runs fit in `slots`, else of the counts
// themselves; in place.  The sums run over an order of the buckets that
// keeps the loads coalesced: thread t owns buckets t, t + 1024, t + 2048,
// ... and the threads' runs follow each other (any order of the buckets
// groups the messages the same way).  One workgroup of 1024 threads: each
// sums its buckets, a wave scans its threads' sums with lane shuffles,
// every thread adds the totals of the waves before its own and reads its
// buckets again to write their starts (kept in registers, the counts would
// spill).  The caller
// keeps the rounded total below 2^32.
__global__ __launch_bounds__(1024) void k_order_scan(unsigned *cnt, unsigned ng, unsigned slots)
{
    constexpr int PER = kBuckets / 1024, WAVES = 1024 / 64;
    __shared__ unsigned wsum[WAVES], wpsum[WAVES];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const unsigned mask = ng - 1u;
    unsigned s = 0u, ps = 0u;
#pragma unroll 16
    for (int k = 0; k < PER; ++k) {
        const unsigned v = cnt[k * 1024 + t];
        s += v;
        ps += (v + mask) & ~mask;
    }
    unsigned is = s, ips = ps;                  // inclusive scans within the wave
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
    unsigned base = 0u, pbase = 0u, ptot = 0u;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) {
        const unsigned a = wsum[k], b = wpsum[k];
        if (k < wv) {
            base += a;
            pbase += b;
        }
        ptot += b;
    }
    const bool pad = ptot <= slots;
    unsigned run = pad ? pbase + ips - ps : base + is - s;
    const unsigned keep = pad ? ~mask : ~0u, add = pad ? mask : 0u;
#pragma unroll 16
    for (int k = 0; k < PER; ++k) {             // the counts again (cached), each replaced by its run's start
        const unsigned v = cnt[k * 1024 + t];
        cnt[k * 1024 + t] = run;
        run += (v + add) & keep;
    }
}

__global__ void k_order_place(const uint32_t *p, const uint32_t *dp, const uint32_t *dq, unsigned long long count,
                              int hl, unsigned *cursor, unsigned *order)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const unsigned at = atomicAdd(&cursor[key_bucket(p, dp, dq, i, hl)], 1u);
    order[at] = (unsigned)i;
}

static hipError_t launch_order(const uint32_t *p, const uint32_t *dp, const uint32_t *dq, size_t count, int hl,
                               size_t ng, size_t slots, unsigned *cnt, unsigned *order, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((count + 255) / 256);
    const size_t fill = slots > (size_t)kBuckets ? slots : (size_t)kBuckets;
    hipLaunchKernelGGL(k_order_clear, dim3((unsigned)((fill + 255) / 256)), dim3(256), 0, stream, cnt, order,
                       (unsigned long long)slots);
    hipLaunchKernelGGL(k_order_count, dim3(blocks), dim3(256), 0, stream, p, dp, dq, (unsigned long long)count, hl,
                       cnt);
    // the rounded runs total at most count + kBuckets * (ng - 1): no rounding
    // where that could pass 2^32
    const unsigned round_to = count + (size_t)kBuckets * ng <= (size_t)0xFFFFFFFFu ? (unsigned)ng : 1u;
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(1024), 0, stream, cnt, round_to, (unsigned)slots);
    hipLaunchKernelGGL(k_order_place, dim3(blocks), dim3(256), 0, stream, p, dp, dq, (unsigned long long)count, hl,
                       cnt, order);
    return hipGetLastError();
}

size_t key_order_slots(size_t count, size_t ng, size_t cus)
{
    const size_t waves = (count + ng - 1) / ng;                       // wave pairs of the dense order
    const size_t round = 2 * (cus ? cus : 1);
    const size_t up = waves <= round / 2 ? round / 2 : (waves + round - 1) / round * round;
    const size_t keys = count < (size_t)kBuckets ? count : (size_t)kBuckets;
    const size_t most = waves + keys;           // the padded runs never take more
    return (up < most ? up : most) * ng;
}

static bool order_args_ok(size_t count, size_t ng, size_t slots)
{
    return ng > 0 && (ng & (ng - 1)) == 0 && slots >= count && slots < (size_t)kOrderHole;
}

// Scratch of the plain CRT call: one buffer per (device, stream handle),
// made on the first call that needs it and grown (doubling) when a larger
// batch arrives; a call therefore allocates only the first time a stream
// sees a batch of its size.  Buffers are never released while the process
// runs: an outgrown buffer is kept, since a HIP graph captured earlier may
// still name it.  Calls on one stream reuse its buffer in stream order;
// calls on distinct streams use distinct buffers.
namespace {
struct StreamScratch {
    int dev;
    hipStream_t stream;
    void *mem;
    size_t bytes;
};
std::mutex g_scratch_mu;
std::vector<StreamScratch> g_scratch;
std::vector<void *> g_outgrown;
}  // namespace

size_t key_order_bytes(size_t slots) { return (slots + kBuckets) * sizeof(unsigned); }

// Scratch of the non-allocating CRT call: static device memory (one copy per
// device, held until the process ends) for the bucket counters and the order
// of up to kStaticOrderMax slots.  Host code never names the array in a
// launch: its device address is looked up once per device (order_static_init)
// and that address is what the kernels receive.  Every call on a device
// shares the array, so such calls must not overlap in time on one device.
static __device__ __align__(256) unsigned scratch[kBuckets + kStaticOrderMax];

namespace {
const int kMaxDev = 64;
unsigned *g_static_order[kMaxDev];
std::mutex g_static_mu;
}  // namespace

int order_static_init(int dev)
{
    if (dev < 0 || dev >= kMaxDev) return -1;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_order[dev]) return 0;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return -1;
    }
    g_static_order[dev] = static_cast<unsigned *>(ptr);
    return 0;
}

unsigned *key_order_static(const uint32_t *p, const uint32_t *dp, const uint32_t *dq, size_t count, int hl,
                           size_t ng, size_t slots, hipStream_t stream)
{
    int dev = 0;
    if (slots > kStaticOrderMax || !order_args_ok(count, ng, slots) || hipGetDevice(&dev) != hipSuccess || dev < 0 ||
        dev >= kMaxDev)
        return nullptr;
    unsigned *cnt = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_static_mu);
        cnt = g_static_order[dev];
    }
    if (!cnt) return nullptr;
    unsigned *order = cnt + kBuckets;
    if (launch_order(p, dp, dq, count, hl, ng, slots, cnt, order, stream) != hipSuccess) return nullptr;
    return order;
}

unsigned *key_order(const uint32_t *p, const uint32_t *dp, const uint32_t *dq, size_t count, int hl, size_t ng,
                    size_t slots, hipStream_t stream)
{
    if (!order_args_ok(count, ng, slots)) return nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    const size_t need = key_order_bytes(slots);
    void *mem = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        StreamScratch *s = nullptr;
        for (StreamScratch &x : g_scratch)
            if (x.dev == dev && x.stream == stream) s = &x;
        if (s && s->bytes >= need) {
            mem = s->mem;
        } else {
            // no allocation while the stream is being captured into a graph:
            // the batch then runs in the given order
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
                (void)hipGetLastError();
                return nullptr;
            }
            const size_t bytes = s && 2 * s->bytes > need ? 2 * s->bytes : need;
            if (hipMalloc(&mem, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            if (s) {
                g_outgrown.push_back(s->mem);
                s->mem = mem;
                s->bytes = bytes;
            } else {
                g_scratch.push_back(StreamScratch{dev, stream, mem, bytes});
            }
        }
    }
    unsigned *cnt = static_cast<unsigned *>(mem), *order = cnt + kBuckets;
    if (launch_order(p, dp, dq, count, hl, ng, slots, cnt, order, stream) != hipSuccess) return nullptr;
    return order;
}

}  // namespace rsagpu
