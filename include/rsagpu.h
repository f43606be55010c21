/*
 * rsagpu.h - C ABI of the MI355X (gfx950) batched RSA modular-exponentiation
 * library (librsagpu.so).
 *
 * The library computes, for many independent messages at once, the RSA
 * transformations C = M^e mod n and M = C^d mod n (paper, Section 2 and
 * Sections 3.2-3.3), one exponentiation per message, all messages in
 * parallel (the data-parallel decomposition of the paper's Section 6).
 *
 * Conventions shared by every entry point:
 *   - A big integer is an array of little-endian 32-bit limbs, limb 0 least
 *     significant.  A batch of `count` integers of `limbs` limbs each is
 *     message-major: element i occupies words [i*limbs, (i+1)*limbs).
 *   - Every data pointer is a DEVICE pointer owned by the caller (for
 *     instance the storage of a torch tensor).  The library never frees or
 *     keeps it past the call's stream work.
 *   - Work is enqueued on `stream` (NULL = the null stream) and is
 *     asynchronous: the call returns before the results exist.  No entry
 *     point synchronises the device except rsa_device_errors.
 *   - Operands and the window table of each exponentiation live in
 *     registers and LDS.  No entry point allocates device memory per call:
 *     rsa_modexp_batch needs no scratch, rsa_ops_batch takes a caller
 *     workspace, and rsa_decrypt_crt_batch keeps one key-ordering buffer per
 *     device and stream handle, made the first time that stream needs one
 *     of its size (see there).  rsa_autotune and rsa_keyset_create allocate
 *     their own buffers.  The per-device error counter is static device
 *     memory.
 *   - Host-checkable errors are returned before any HIP call.  Per-element
 *     data errors (an even or unit modulus, p <= q for CRT) write 0 to that
 *     element's output and increment a per-device counter that
 *     rsa_device_errors reads.
 *   - The ABI is thread-safe for calls on distinct streams.  Results are
 *     exact: every output is the unique residue in [0, modulus).
 */
#ifndef RSAGPU_H
#define RSAGPU_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSA_OK = 0,
    RSA_EINVAL = -1,   /* null pointer, bad count or bad option            */
    RSA_ELIMBS = -2,   /* limb width outside the supported range           */
    RSA_ENOMEM = -3,   /* device memory exhausted                          */
    RSA_EHIP = -4,     /* a HIP runtime call failed                        */
    RSA_EKEY = -5      /* malformed key material                           */
} rsa_status;

/* Largest limb width accepted (4096-bit operands). */
#define RSA_MAX_LIMBS 128

/*
 * Batched modular exponentiation (paper, Section 2: C = M^e mod n; the same
 * operation with d decrypts, Section 11).
 *
 *   out[i] = base[i] ^ exp[i] mod mod[i],   0 <= i < count
 *
 * base, exp, mod, out: count * limbs words each (device, message-major).
 * base may be >= mod (it is reduced); exp == 0 gives 1 mod n.  Every mod[i]
 * must be odd and > 1 (Montgomery arithmetic); an even modulus, or a
 * modulus equal to 1, is a data error (output 0, counter incremented;
 * for mod == 1 the output 0 is also the correct value and is not counted).
 * out may be the same buffer as base; other overlap is undefined.
 * 1 <= limbs <= RSA_MAX_LIMBS; count == 0 is a no-op returning RSA_OK.
 * Montgomery constants are derived per element on the device; for many
 * messages under one key prefer the resident-key entry points (keyset).
 */
int rsa_modexp_batch(const uint32_t *base, const uint32_t *exp, const uint32_t *mod,
                     uint32_t *out, size_t count, int limbs, hipStream_t stream);

/*
 * Batched RSA decryption by the Chinese remainder theorem.
 *
 *   out[i] = c[i] ^ d mod (p[i] * q[i])
 *
 * computed as m_p = c^dp mod p and m_q = c^dq mod q followed by Garner's
 * recombination m = m_q + q * (qinv * (m_p - m_q) mod p).  The result equals
 * the paper's plain decryption M = C^d mod n (Section 2) for every
 * c in [0, n) when d*e = 1 mod phi(n) and dp = d mod (p-1), dq = d mod (q-1).
 *
 * c, out: count * limbs words; p, q, dp, dq, qinv: count * (limbs/2) words
 * (device, message-major).  limbs is the width of the modulus n = p*q and
 * must be even, 2 <= limbs <= RSA_MAX_LIMBS.  Convention p > q and
 * qinv = q^-1 mod p; p, q odd and > 1.  Violations are data errors.
 * c must be < p*q (it is the caller's ciphertext).
 * Messages under the same key are processed together (one exponent per
 * wave): for more than one wave's worth of messages the call orders them by
 * a hash of their key words, each key's run starting a wave of its own where
 * the padding adds no round of waves to the launch, in a scratch buffer
 * (4 bytes per slot of that order, the batch rounded up to whole waves and
 * at most 2 waves per CU more, + 256 KiB) that the library keeps for the
 * current device and this stream handle.  The first call on a stream, and a call with a larger
 * batch than that stream has seen, allocates it (hipMalloc; an outgrown
 * buffer is kept until the process ends, so graphs captured earlier stay
 * valid); later calls allocate nothing.  While `stream` is being captured
 * into a graph the call never allocates: without a large enough buffer the
 * batch runs in the given order (warm a stream up before capturing on it).
 * If an allocation fails the batch also runs in the given order.  The order
 * never changes a result.  Calls on distinct streams use distinct buffers;
 * calls on one stream are ordered by the stream.
 */
int rsa_decrypt_crt_batch(const uint32_t *c, const uint32_t *p, const uint32_t *q,
                          const uint32_t *dp, const uint32_t *dq, const uint32_t *qinv,
                          uint32_t *out, size_t count, int limbs, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation and arguments as rsa_decrypt_crt_batch, with identical results,
 * but the key-ordering scratch is the library's static device array (one
 * copy per device, ~4.25 MiB, held until the process ends), so the call
 * never allocates, whatever the stream or batch size.
 * count <= RSA_CRT_STATIC_MAX_COUNT (RSA_EINVAL beyond, before any HIP call).
 * Every call on a device shares that array: calls that overlap in time on
 * one device (on different streams, or from different threads) race and
 * may give wrong results; serialise them, for instance on one stream.
 * Each call clears what it uses with a kernel (no memset), so it may be
 * captured into a graph and replayed.  Returns RSA_EHIP if the array's
 * device address cannot be looked up or a launch fails.
 */
#define RSA_CRT_STATIC_MAX_COUNT 1048576
int rsa_decrypt_crt_batch_static(const uint32_t *c, const uint32_t *p, const uint32_t *q,
                                 const uint32_t *dp, const uint32_t *dq, const uint32_t *qinv,
                                 uint32_t *out, size_t count, int limbs, hipStream_t stream);

/*
 * Execution plan used for a limb width: the limb radix the kernel computes
 * in (radix_bits = 32, or 29 for the reduced-radix kernels whose 64-bit
 * accumulators need no carry handling), the kernel's limb count in that
 * radix (padded_limbs), lanes per exponentiation (G), limbs per lane
 * (padded_limbs / G), window width in exponent bits (a sliding window over
 * the 2^(window_bits-1) odd powers, paper Section 3.6.5) and the LDS bytes
 * per wave.  The CRT kernels run a wave per half, in workgroups of one
 * pair of waves, or of two pairs (one wave per SIMD of a CU): in
 * rsa_decrypt_crt_batch (kind 1) where lanes_per_op is 8 or 16, and for
 * fewer lanes in calls that need one to two one-pair workgroups per CU; in
 * every CRT bucket of a bulk rsa_ops_batch call (at least 16384
 * operations); each only where the LDS holds two pairs.  A workgroup takes
 * 2 or 4 times lds_bytes.
 * kind: 0 = plain exponentiation (rsa_modexp_batch), 1 = CRT half
 * (rsa_decrypt_crt_batch, modulus of `limbs` limbs), 2 and 3 = the same
 * operations inside rsa_ops_batch (separate plans: its buckets are smaller
 * and run side by side), 4 = the CRT half of the widest class of an
 * rsa_ops_batch call with at least 16384 operations (the bucket that ends
 * such a batch).
 * Inputs and outputs are 32-bit limbs whatever the radix.  Pure host query.
 */
typedef struct {
    int radix_bits;
    int padded_limbs;
    int lanes_per_op;
    int limbs_per_lane;
    int window_bits;
    int lds_bytes;
} rsa_plan;

int rsa_get_plan(int limbs, int kind, rsa_plan *plan);

/*
 * Overrides the plan of the width class that `limbs` maps to (kind as in
 * rsa_get_plan): (radix_bits, lanes_per_op) must name a compiled kernel
 * instance for that class, 2 <= window_bits <= 7, and the plan's LDS
 * (lds_bytes of rsa_get_plan) must fit 64 KiB; for a CRT kind (1, 3, 4) the
 * workgroup's LDS (2 or 4 times lds_bytes, as above, plus 16 bytes) must
 * also fit the 160 KiB a workgroup may hold.  All three zero restores the
 * default.
 * Used by the tuner; affects calls issued afterwards from any thread.
 * Pure host call.
 */
int rsa_set_plan(int limbs, int kind, int radix_bits, int lanes_per_op, int window_bits);

/*
 * Autotuner: for the width class of `limbs` and plan `kind` (as in
 * rsa_get_plan), times every compiled kernel instance of the class at every
 * window width that fits, on `count` synthetic operands laid out as the
 * workloads have them, and installs the fastest plan (rsa_set_plan):
 *   kind 0: rsa_modexp_batch of `limbs`-word operands under one modulus and
 *           one exp_bits-bit exponent (one key's messages);
 *   kind 1: rsa_decrypt_crt_batch of `limbs`-word moduli, 16 keys
 *           round-robin, exp_bits-bit dp and dq;
 *   kind 2, 3, 4: rsa_ops_batch on a temporary keyset of 16 synthetic keys of
 *           `limbs` words (limbs even), `count` operations round-robin over
 *           the keys: e = 65537 encryptions (kind 2) or CRT decryptions with
 *           full-length dp, dq (kinds 3 and 4; both plans hold the candidate
 *           while it is timed, and the other kind's plan is restored after).
 * exp_bits <= 0 means full length.  count <= 2^22 (kinds 2-4: 2^20).
 * Allocates and frees its own device buffers (and keyset) and synchronises
 * `stream`; not for use inside a timed or captured region.  The chosen
 * plan is written to *best when not NULL.
 */
int rsa_autotune(int limbs, int kind, int exp_bits, size_t count, hipStream_t stream, rsa_plan *best);

/*
 * Sets up the current device's library state (looks up the addresses of
 * the data-error counter and of rsa_decrypt_crt_batch_static's scratch,
 * both static device memory; allocates nothing).  Every other entry point
 * does this on first use.
 */
int rsa_init(void);

/* ---- resident keys and mixed batches ------------------------------------
 *
 * A keyset holds RSA keys on the device together with their Montgomery
 * constants (R mod m and R^2 mod m of n, p and q in every limb radix the
 * kernels use), computed once when a key is added, so an operation starts
 * directly with its exponentiation.  A batch is a device array of operation
 * descriptors over keys of any sizes, run by one call: the operations are
 * sorted on the device into buckets of one width class and kind, and each
 * bucket is served by a persistent kernel whose waves claim operations from
 * an atomic counter until the bucket is empty (largest classes first).
 */
typedef struct rsa_keyset rsa_keyset;

typedef struct {
    uint32_t kind;      /* 0: out = in^e mod n; 1: out = in^d mod n by CRT  */
    int32_t key_id;     /* from rsa_keyset_add                               */
    uint64_t in_off;    /* word offset of the input (the key's limbs words)  */
    uint64_t out_off;   /* word offset of the output (same width)            */
} rsa_op;

/* Creates an empty keyset for up to max_keys keys on the current device.
 * Allocates the keyset's device memory once (~8.3 KB per key). */
int rsa_keyset_create(rsa_keyset **ks, int max_keys);

/*
 * Adds a key (HOST pointers, synchronous): n and e have `limbs` words,
 * p, q, dp, dq, qinv have limbs/2 words; limbs even, 2 <= limbs <= 128.
 * Checks n odd, p > q, p and q odd, n = p*q and e != 0 (RSA_EKEY otherwise),
 * uploads the material and computes the Montgomery constants on the device.
 * Not safe concurrently with rsa_ops_batch on the same keyset.
 */
int rsa_keyset_add(rsa_keyset *ks, int limbs, const uint32_t *n, const uint32_t *e, const uint32_t *p,
                   const uint32_t *q, const uint32_t *dp, const uint32_t *dq, const uint32_t *qinv,
                   int32_t *key_id);

/* Frees the keyset (synchronises the device first). */
int rsa_keyset_destroy(rsa_keyset *ks);

/* Bytes of workspace rsa_ops_batch needs for up to max_ops operations. */
size_t rsa_ops_workspace_size(size_t max_ops);

/*
 * Runs nops operations (device array `ops`) against the keyset: for each op,
 * out_pool[out_off ..] = in_pool[in_off ..]^(e or d) mod n of its key, each
 * range the key's limbs words; the input must be < n.  in_words / out_words
 * bound the pools: an operation whose kind, key id or ranges are invalid is
 * skipped and counted as a data error.  workspace: caller-owned device
 * memory of at least rsa_ops_workspace_size(nops) bytes; calls that overlap
 * in time must use different workspaces.  nops < 2^32 (RSA_EINVAL beyond).
 * Asynchronous on `stream`.
 */
int rsa_ops_batch(rsa_keyset *ks, const rsa_op *ops, size_t nops, const uint32_t *in_pool, size_t in_words,
                  uint32_t *out_pool, size_t out_words, void *workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Streams an rsa_ops_batch call forks its widest CRT buckets onto (0 to 3,
 * default 3), beside the caller's stream, which runs every other bucket and
 * then waits for the forks.  Each caller stream has a fork set of its own
 * (up to 8 caller streams per keyset; further callers, and a caller first
 * seen while it is being captured into a graph, run unforked), so calls on
 * different caller streams overlap on the device.  A process has 4 hardware
 * queues and streams beyond them share queues and serialise, so callers x
 * (forks + 1) <= 4 keeps every bucket concurrent: 3 for one caller, 1 for
 * two, 0 (every bucket in order on the caller's stream) for more.  Results
 * do not depend on it.  Pure host setting, applies to later calls.
 */
int rsa_keyset_set_forks(rsa_keyset *ks, int forks);

/*
 * Number of per-element data errors counted on the current device since the
 * last call, reset to zero in the same atomic step (a one-thread kernel on
 * `stream`), so counts added later, by work on any stream, go to the next
 * call.  Synchronises `stream` (only) and returns the count.
 */
int rsa_device_errors(hipStream_t stream, uint64_t *n_bad);

/* Static text for a status code. */
const char *rsa_status_str(int status);

/* ABI version (major * 10000 + minor * 100 + patch). */
int rsa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RSAGPU_H */
