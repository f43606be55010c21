// Host-side registry shared by the C-ABI translation units: kernel instances,
// width classes, execution plans and per-device state.
#pragma once

#include "launch.hpp"

namespace rsagpu {

struct Instance {
    int B;
    int S;
    int G;
    modexp_launcher modexp;
    crt_launcher crt;
    setup_launcher setup;
    ops_launcher ops_enc;
    ops_launcher ops_crt;
    ops_launcher ops_crt_pairs;       // two pairs per workgroup (the CRT buckets of a bulk batch)
    ops_occupancy blocks_per_cu;
};

// Width classes in 32-bit limbs and their radix-2^29 limb counts.
int num_classes();
int class_width(int i);
int class_s29(int i);
int class_index(int limbs);

// Instance of class i in radix 2^B with G lanes per exponentiation.
const Instance *find_instance(int i, int B, int G);
// Any instance of class i in radix 2^B (for work whose speed does not matter).
const Instance *any_instance(int i, int B);

struct Resolved {
    const Instance *inst;
    int w;
};
bool resolve(int limbs, int kind, Resolved *r);
// rsa_ops_batch calls of at least this many operations take the kind-4 plan
// for the CRT bucket of their widest class.
static const size_t kBulkOps = 16384;

// Processing order of a plain CRT batch that puts messages under the same key
// next to each other: a device array of `slots` entries, each a message index
// or kOrderHole, every one of the count messages in exactly one; nullptr to
// keep the given order.  ng (a power of two) is the messages of one wave;
// each key's run starts a wave when the runs so rounded up fit in the slots.
// key_order_slots gives the slots to ask for on a device of `cus` compute
// units: the dense order's wave pairs rounded up to cus (one pair per CU) if
// they fit in that, else to a multiple of 2 cus (one wave per SIMD), so that
// the padding does not change the launch's shape, and never more than the
// padded runs can take.  The scratch (key_order_bytes(slots))
// is the library's buffer for this device and stream handle, made or grown
// on first need (never while the stream is being captured: the given order
// is kept then).
size_t key_order_slots(size_t count, size_t ng, size_t cus);
size_t key_order_bytes(size_t slots);
unsigned *key_order(const uint32_t *p, const uint32_t *dp, const uint32_t *dq, size_t count, int hl, size_t ng,
                    size_t slots, hipStream_t stream);

// The same order in the library's static device scratch (no allocation):
// order_static_init looks up the scratch's address on device `dev` (once per
// device, 0 on success); key_order_static then returns the order in up to
// kStaticOrderMax slots, or nullptr (not set up, too many slots, or a launch
// failure).  Calls on one device share the scratch.
static const size_t kStaticOrderMax = (size_t)1 << 20;
int order_static_init(int dev);
unsigned *key_order_static(const uint32_t *p, const uint32_t *dp, const uint32_t *dq, size_t count, int hl,
                           size_t ng, size_t slots, hipStream_t stream);

// Per-device data-error counter: two words of static device memory (the
// count, and the value rsa_device_errors last took), looked up once per device.
// device_state also gives the current device's compute units (cus, if not
// null).
int device_state(unsigned long long **errs, int *cus = nullptr);
int status_of(hipError_t e);

}  // namespace rsagpu
