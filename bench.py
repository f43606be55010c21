#!/usr/bin/env python3
"""Benchmark: batched RSA modular exponentiation on one MI355X.

Default workload (the headline metric): 2048-bit RSA, 64 seeded keys, 16384
messages assigned round-robin, CRT decryption (two 1024-bit exponentiations
with dp, dq and Garner recombination per message).  One step = one CRT-
decryption pass over the whole batch with inputs resident in HBM.  The JSON
line carries

  roofline:     the decryption kernel against the chip's 32x32-bit integer
                multiply peak (256 CUs x 64 lanes x 2.4 GHz, one
                v_mad_u64_u32 per lane per clock).  `achieved` counts the
                method's algorithmic products per unit - the k-ary method of
                Section 3.6.4 at the window that minimises them, every
                squaring a general Montgomery product of 2s^2 + s 32x32-bit
                products, conversions included, and for CRT the two
                reductions of c and Garner's recombination - times the units
                of one launch, over the mean step time from HIP events on the
                launch stream.  `as_run` gives the tighter count of the
                schedule the kernel runs (sliding window, symmetric
                squarings), `peak_measured` the multiply rate the probe
                library sustains in the same run;
  cpu_baseline: the plain CPU oracle (C^d mod n, no CRT) on the host's
                cores, over the whole batch (every GPU output compared), and
                on one thread over a fixed 256-message prefix;
  latency_ms:   p50 and p99 request latency of a short serving run
                (Poisson arrivals at 0.7 x the saturated rate, 2048/4096-bit
                keys, 70% CRT decryptions); batch_ms: p50/p99 of the whole-
                batch step time;
  check:        elements of the whole batch whose round trip through the
                opposite operation (decryptions re-encrypted, encryptions
                decrypted) differs; the run fails unless it is 0;
  encrypt:      the same batch's messages encrypted with e = 65537, with its
                own rate, roofline, check and oracle comparison.

Other workloads (--workload): crt4096 (the plain CRT call on 4096-bit keys:
16 keys, by default 1092 messages), rsa64, rsa1024 (full-d decryption, no CRT,
and under `encrypt` the same messages' e = 65537 encryptions), enc2048
(e = 65537 encryption of the default batch), mixed (32768 operations
over 1024..4096-bit keys in one rsa_ops_batch call), serve (Poisson requests
through the continuous-batching server: p50/p99 latency and throughput),
paper (the paper's own Section 10 experiment: one-word keys n = 131*137 and
1009*509, e = 131, messages 0..800 at every data size of Tables 1 and 2,
beside the times the tables print, whose unit the paper leaves unclear),
keygen (4096-bit key generation with the Miller-Rabin rounds on the GPU),
mulpeak (the issue rate of the 32-bit integer multiplies, libmulpeak.so).
"""
import argparse
import json
import os
import sys
import time

# Hardware queues per process: a mixed batch runs its widest CRT buckets on
# up to three streams forked from the caller's, and the server keeps two
# batches in flight, each with its forks; streams beyond the queues share
# them and serialise in submission order (HIP's default is 4, one of them
# the null stream's).  Raised to 8 before the runtime starts, unless the
# environment asks for more.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 256 CUs x 64 lanes x 2.4 GHz: one 32x32->64-bit product (v_mad_u64_u32) per
# lane per clock at the full VALU rate.
INT32_MUL_PEAK = 256 * 64 * 2.4e9
METRIC = "2048-bit modexp/sec (CRT decrypt) on 1 GPU, %INT32-mul peak; p50/p99 latency"


def sliding_window_counts(e: int, w: int):
    """(squarings, table products, table size) of the left-to-right sliding
    window over odd powers for exponent e: one squaring per bit below the
    leading window, one product per further window (a window ends in a one
    bit and spans at most w bits), and a table of 2^(w-1) odd powers (for
    exponents of at most 64 bits only up to the largest power used) built
    with x^2 and one product per further entry."""
    if e == 0:
        return 0, 0, 0
    pos, sq, mul, first, used = e.bit_length() - 1, 0, 0, True, 0
    while pos >= 0:
        if not (e >> pos) & 1:
            sq, pos = sq + 1, pos - 1
            continue
        lo = max(pos - w + 1, 0)
        while not (e >> lo) & 1:
            lo += 1
        used = max(used, ((e >> lo) & ((1 << (pos - lo + 1)) - 1)) // 2 + 1)
        if not first:
            sq, mul = sq + pos - lo + 1, mul + 1
        first, pos = False, lo - 1
    tsize = (1 << (w - 1)) if e.bit_length() > 64 else used
    return sq, mul, tsize


def sliding_window_montmuls(e: int, w: int) -> int:
    """Montgomery products (squarings included) of one exponentiation."""
    sq, mul, tsize = sliding_window_counts(e, w)
    return sq + mul + (tsize if tsize > 1 else 0)


def mont_products(s: int) -> int:
    """32x32-bit products of one Montgomery product of s 32-bit limbs:
    s^2 for a*b, s^2 for m*n, s for the m_i."""
    return 2 * s * s + s


def sqr_products(s: int) -> int:
    """32x32-bit products of one Montgomery squaring of s 32-bit limbs when
    each pair of limbs is multiplied once: s(s+1)/2 for a^2, s^2 + s for the
    reduction."""
    return s * (s + 1) // 2 + s * s + s


def symmetric_squarings(plan) -> bool:
    """Whether the plan's kernel squares with one product per limb pair:
    radix 2^29 with at most 20 limbs per lane.  Its waves do so when all
    their exponents are equal (one key, or a public exponent); the count
    below credits every squaring at the symmetric cost, so a wave that
    mixes exponents is charged less than it computes."""
    return plan.radix_bits == 29 and 3 * plan.limbs_per_lane <= 62


def exp_products(e: int, plan, s: int, general_squarings: bool = False) -> int:
    """Algorithmic 32x32-bit products of x^e mod n at s 32-bit limbs with
    the plan's window (general_squarings: every squaring counted as a
    general product, for comparison)."""
    sq, mul, tsize = sliding_window_counts(e, plan.window_bits)
    sym = symmetric_squarings(plan) and not general_squarings
    per_sq = sqr_products(s) if sym else mont_products(s)
    return sq * per_sq + (mul + (tsize if tsize > 1 else 0)) * mont_products(s)


def per_key_sum(key_of, fn) -> int:
    """sum(fn(k) for k in key_of), evaluating fn once per distinct key."""
    import collections
    keys = key_of.tolist() if hasattr(key_of, "tolist") else key_of
    return sum(n * fn(k) for k, n in collections.Counter(map(lambda x: tuple(x) if isinstance(x, list) else x,
                                                             keys)).items())


def crt_products(key, plan, general_squarings: bool = False) -> int:
    """Two half exponentiations and Garner's product (h^2 more for m_q + h*q)."""
    h = key.limbs // 2
    return (exp_products(key.dp, plan, h, general_squarings) + exp_products(key.dq, plan, h, general_squarings) +
            mont_products(h) + h * h)


def modexp_products(key, e: int, plan) -> int:
    return exp_products(e, plan, key.limbs)


# ---- the method's algorithmic products per unit (k-ary count) --------------

def kary_montmuls(bits: int):
    """(T, w): Montgomery products of one exponentiation with a `bits`-bit
    exponent by the k-ary method (Section 3.6.4, Fig. 6) at the window w that
    minimises T = (ceil(bits/w) - 1)(w + 1) + 2^w: w squarings and one table
    product per further digit, and 2^w for the table of powers x^0 .. x^(2^w-1)
    with the conversions into and out of Montgomery form."""
    return min(((-(-bits // w) - 1) * (w + 1) + (1 << w), w) for w in range(1, 12))


def unit_exp_products(s: int, bits: int = 0) -> int:
    """32x32-bit products of x^d mod n, n and d of s 32-bit limbs (full-length
    d unless `bits` is given), every squaring a general product."""
    return kary_montmuls(bits or 32 * s)[0] * mont_products(s)


def unit_enc_products(s: int) -> int:
    """The same for e = 65537 by the binary method of Fig. 5: 16 squarings,
    one product and the two conversions."""
    return 19 * mont_products(s)


def unit_crt_products(h: int) -> int:
    """One CRT decryption of a 2h-limb modulus: per half the reduction of c
    (h^2 + h) and a full-length h-limb exponentiation, then Garner's
    recombination (a Montgomery product and the h x h product h*q)."""
    return 2 * (unit_exp_products(h) + h * h + h) + mont_products(h) + h * h


# ---- host and probe ----------------------------------------------------------

def host_cpus():
    """(cpus this process may run on, logical CPUs of the host, CPU model):
    the first is the affinity set, lowered to the cgroup quota if one is set."""
    n = os.cpu_count() or 1
    share = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else n
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            quota, period = f.read().split()[:2]
        if quota != "max":
            share = max(1, min(share, -(-int(quota) // int(period))))
    except (OSError, ValueError):
        pass
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return share, n, model


def oracle_threads():
    """Threads for the CPU oracle: the CPUs this process may use, at most 16
    (the CPU share that goes with one GPU on the machines this runs on)."""
    return min(16, host_cpus()[0])


def measured_peak(quick: bool = True):
    """v_mad_u64_u32 issue rate from the probe library (products/s), or None."""
    try:
        from paper_1407_1465_amd import mulpeak
        r = mulpeak.measure(0, iters=4096 if quick else 8192, reps=3 if quick else 7)
    except (ImportError, RuntimeError, OSError) as e:
        print("# multiply probe unavailable: %s" % e, file=sys.stderr, flush=True)
        return None
    return r


def timed(fn, steps, warmup, torch, per_step=None):
    """Mean ms per step over `steps` back-to-back steps (HIP events on the
    launch stream); per_step, if a list, receives each step's ms."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    wall0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(steps):
        fn()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    if per_step is not None:
        per_step.extend(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    return evs[0].elapsed_time(evs[-1]) / steps, time.perf_counter() - wall0


def row_mismatches(a, b) -> int:
    """Rows (elements) of two (count, limbs) device tensors that differ."""
    return int((a != b).any(dim=1).sum().item())


def percentile(xs, q):
    """q-th percentile (nearest rank) of a non-empty list."""
    ys = sorted(xs)
    return ys[min(len(ys) - 1, max(0, int(-(-q * len(ys) // 100)) - 1))]


# Sources the plain exponentiation and CRT kernels are compiled from (device
# arithmetic, kernels, launch configuration); host-only files are left out.
KERNEL_SOURCES = ("group_bn.hpp", "radix_bn.hpp", "modexp_kernels.hpp", "launch.hpp", "launch_impl.hpp")


def kernel_src_hash():
    """sha256 over the sources the plain kernels are built from."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1407_1465_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter profile of `kernel`
    (FETCH_SIZE and WRITE_SIZE runs scaled by a plain copy of known size), or
    None when there is none or the sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "k_crt_rsa2048_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel") != kernel.replace(" ", "") or t.get("src_sha256") != kernel_src_hash():
        return None
    return t.get("traffic_bytes_per_launch")


def roofline(products, ms, kernel, per_unit=None, units=None, as_run=None, peak=None):
    """Roofline object of the dominant kernel: `products` algorithmic 32x32-bit
    products per launch (per_unit x units) over `ms` per launch; `as_run` the
    products of the schedule the kernel runs (for its fraction beside);
    `peak` the probe's measured multiply rate."""
    achieved = products / (ms / 1e3)
    r = {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_MUL_PEAK / 1e12,
         "unit": "T int32-mul/s", "frac": achieved / INT32_MUL_PEAK, "traffic": measured_traffic(kernel),
         "kernel": kernel, "products_per_launch": products, "products_per_unit": per_unit,
         "units_per_launch": units, "ms_per_launch": ms}
    if as_run is not None:
        r["as_run"] = {"products_per_launch": as_run, "frac": as_run / (ms / 1e3) / INT32_MUL_PEAK,
                       "count": "sliding window as run, squarings at the symmetric cost where the kernel "
                                "squares with one product per limb pair"}
    if peak is not None:
        r["peak_measured"] = {"value": peak["ops_per_s"] / 1e12, "unit": "T int32-mul/s", "op": peak["op"],
                              "frac_of_nominal": peak["ops_per_s"] / INT32_MUL_PEAK}
        r["frac_of_measured_peak"] = achieved / peak["ops_per_s"]
    return r


def cpu_baseline(oracle, base, exp, mod, gpu_out, unit, what, count=None, prefix=256):
    """The oracle on the host's cores over the first `count` elements (all by
    default), every output compared with the GPU's, and on one thread over the
    first `prefix` elements."""
    import numpy as np
    share, ncpu, model = host_cpus()
    threads = oracle_threads()
    n = len(base) if count is None else min(count, len(base))
    k = min(prefix, n)
    one, wall1, _ = oracle.modexp_batch(base[:k], exp[:k], mod[:k], nthreads=1)
    c0 = time.process_time()
    got, cwall, used = oracle.modexp_batch(base[:n], exp[:n], mod[:n], nthreads=threads)
    ccpu = time.process_time() - c0
    bad = int((got != gpu_out[:n]).any(axis=1).sum())
    if bad or not np.array_equal(one, got[:k]):
        raise SystemExit("GPU output differs from the oracle on %d of %d elements" % (bad, n))
    return {"value": n / cwall, "unit": unit, "cores": used, "kind": "oracle",
            "sample": "%s %d elements of the same batch, %s, %.1f s wall, %.1f s CPU; every output equals "
                      "the GPU's" % ("all" if n == len(base) else "the first", n, what, cwall, ccpu),
            "verified": n, "mismatches": bad, "cpu_model": model, "host_cpus": ncpu, "cpu_share": share,
            "one_thread": {"value": k / wall1, "unit": unit, "sample": "first %d elements" % k}}


def serve_leg(torch, np, rsagpu, W, seconds, plain_requests=0, streams=2, forks=3):
    """Serving run (256 x 2048-bit + 64 x 4096-bit resident keys, 70% CRT
    decryptions, 1..256 messages per request): the saturated request rate as
    the median of three closed bursts of 400 requests (after one unmeasured
    burst), then Poisson arrivals at 0.7 x that rate for `seconds`; every
    served message checked through the opposite operation afterwards.  With
    plain_requests > 0 also the rate of the plain form: the same kind of
    requests, one launch of the plain entry points per request (device-
    resident inputs, no host copies), back to back on one stream."""
    from paper_1407_1465_amd.serve import GpuExecutor, Server, poisson_requests
    keys = W.make_keys(2048, W.SEED_BASE + 5, 256) + W.make_keys(4096, W.SEED_BASE + 5, 64)
    ks = rsagpu.KeySet(len(keys))
    for k in keys:
        ks.add(k.limbs, k.n, k.e, k.p, k.q, k.dp, k.dq, k.qinv)
    limbs = [k.limbs for k in keys]
    mods = [k.n for k in keys]
    pool, max_ops = 1 << 23, 1 << 16
    ex = GpuExecutor(ks, limbs, pool, max_ops, streams=streams, forks=forks)
    last = {}

    def run(reqs):
        srv = Server(ex, pool, max_inflight=ex.max_inflight, max_ops=max_ops)
        srv.run(reqs)
        last["finished"] = srv.finished
        return srv.stats()

    def verify(finished):
        items = [(r.kind, r.key_id, row) for r in finished if r.error is None
                 for row in zip(r.outputs, r.inputs)]
        bad, chunk = 0, 1 << 15
        ws_v = torch.empty(rsagpu.ops_workspace_size(chunk), dtype=torch.uint8, device="cuda")
        for i0 in range(0, len(items), chunk):
            part = items[i0:i0 + chunk]
            offs = np.cumsum([0] + [limbs[kid] for _, kid, _ in part])
            outs = np.concatenate([o for _, _, (o, _) in part]).astype(np.uint32)
            ins = np.concatenate([x for _, _, (_, x) in part]).astype(np.uint32)
            vops = rsagpu.pack_ops(np.array([1 - k for k, _, _ in part]), np.array([kid for _, kid, _ in part]),
                                   offs[:-1], offs[:-1]).cuda()
            back = torch.zeros(int(offs[-1]), dtype=torch.int32, device="cuda")
            rsagpu.ops_batch(ks, vops, _dev(torch, np, outs), back, ws_v)
            diff = back.cpu().numpy().view(np.uint32) != ins
            bad += int(np.logical_or.reduceat(diff, offs[:-1]).sum())
        return bad, len(items)

    def req_products(r):
        k = keys[r.key_id]
        return len(r.inputs) * (unit_crt_products(k.limbs // 2) if r.kind else unit_enc_products(k.limbs))

    run(poisson_requests(0.0, 400, W.SEED_BASE + 49, limbs, mods))
    bursts = sorted((run(poisson_requests(0.0, 400, W.SEED_BASE + 50 + 10 * i, limbs, mods))
                     for i in range(3)), key=lambda b: b["requests_per_s"])
    sat = bursts[1]
    rate = 0.7 * sat["requests_per_s"]
    nreq = max(200, int(rate * seconds))
    st = run(poisson_requests(rate, nreq, W.SEED_BASE + 51, limbs, mods))
    finished = last["finished"]
    bad, nmsg = verify(finished)
    errs = rsagpu.device_errors()
    products = sum(req_products(r) for r in finished if r.error is None)
    out = {"requests_per_s": st["requests_per_s"], "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
           "mean_ms": st["mean_ms"], "ops_per_s": st["ops_per_s"], "requests": st["requests"],
           "rate_req_per_s": rate, "saturated_req_per_s": sat["requests_per_s"],
           "saturation_bursts_req_per_s": [b["requests_per_s"] for b in bursts], "span_s": st["span_s"],
           "streams": len(ex.streams), "forks": forks, "max_inflight": ex.max_inflight,
           "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
           "check": {"mismatches": bad + st["errors"] + errs,
                     "of": "all %d served messages through the opposite operation, plus failed requests "
                           "and device data errors" % nmsg},
           "products": products}
    if plain_requests:
        reqs = poisson_requests(0.0, plain_requests, W.SEED_BASE + 52, limbs, mods)
        launches = []
        for r in reqs:
            k = keys[r.key_id]
            L, h, cnt = k.limbs, k.limbs // 2, len(r.inputs)
            x = _dev(torch, np, r.inputs)
            if r.kind:
                args = [_dev(torch, np, np.tile(W.int_to_limbs(getattr(k, a), h), (cnt, 1)))
                        for a in ("p", "q", "dp", "dq", "qinv")]
                launches.append(("crt", x, args, torch.empty_like(x)))
            else:
                args = [_dev(torch, np, np.tile(W.int_to_limbs(getattr(k, a), L), (cnt, 1))) for a in ("e", "n")]
                launches.append(("enc", x, args, torch.empty_like(x)))

        def plain():
            for kind, x, args, o in launches:
                if kind == "crt":
                    rsagpu.decrypt_crt(x, *args, out=o)
                else:
                    rsagpu.modexp(x, *args, out=o)
        ms_plain, _ = timed(plain, 2, 1, torch)
        out["plain_one_request_per_launch"] = {"requests_per_s": len(reqs) / (ms_plain / 1e3),
                                               "requests": len(reqs), "ms": ms_plain}
    ks.close()
    return out


def _dev(torch, np, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="crt2048",
                    choices=["crt2048", "crt4096", "rsa64", "rsa1024", "enc2048", "mixed", "serve", "paper", "keygen",
                             "mulpeak"])
    ap.add_argument("--count", type=int, default=0, help="messages (0: the workload's size)")
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="elements the CPU oracle processes for the baseline (-1: the whole batch, 0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=None,
                    help="length of the Poisson serving run (serve: 8 s; the default workload adds a 3 s run "
                         "for its request latencies, 0 leaves it out)")
    ap.add_argument("--no-tune", action="store_true", help="mixed: keep the default plans (no autotuning)")
    ap.add_argument("--plan", action="append", default=[], metavar="WIDTH:KIND:RADIX:LANES:WINDOW",
                    help="set a plan before running (rsa_set_plan; repeatable)")
    ap.add_argument("--serve-streams", type=int, default=2, help="serving: executor streams (batches in flight)")
    ap.add_argument("--serve-forks", type=int, default=None,
                    help="serving: streams each batch forks its widest CRT buckets onto (default: 3 with at "
                         "least 8 hardware queues, else 1)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size reference "
                         "dispatch for hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (operations are independent; "
              "a batch would shard by contiguous ranges with no exchange step)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1407_1465_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build()
    from paper_1407_1465_amd import rsagpu
    from paper_1407_1465_amd import workloads as W
    torch.cuda.set_device(0)
    for spec in args.plan:
        width, kind, radix, lanes, window = (int(v) for v in spec.split(":"))
        rsagpu.set_plan(width, kind, radix, lanes, window)
    if args.plan:
        line_plans = args.plan
    else:
        line_plans = None
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()

    def tab(wl, attr, width):
        return np.ascontiguousarray(W.ints_to_limbs([getattr(k, attr) for k in wl.keys], width)[wl.key_of])

    def encrypt_half(wl, L, n_h, e_h, decrypt):
        """The batch's other half: every message encrypted (e = 65537) with
        its key, timed like the line's own operation, each output decrypted
        back (`decrypt`) against its message and, with the CPU baseline on,
        compared with the oracle's."""
        m, e, n = dev(wl.msgs), dev(e_h), dev(n_h)
        out = torch.empty_like(m)
        plan = rsagpu.get_plan(L, 0)
        count = len(wl.msgs)
        ms_e, _ = timed(lambda: rsagpu.modexp(m, e, n, out=out), args.steps, args.warmup, torch)
        bad = row_mismatches(decrypt(out), m)
        if bad:
            raise SystemExit("encryption round trip failed on %d elements" % bad)
        per_unit = unit_enc_products(L)
        as_run = per_key_sum(wl.key_of, lambda k: modexp_products(wl.keys[k], wl.keys[k].e, plan))
        sub = {"value": count / (ms_e / 1e3), "unit": "encryptions/s", "ms_per_step": ms_e,
               "roofline": roofline(per_unit * count, ms_e, "k_modexp<%d,%d,%d>" % (
                   plan.padded_limbs, plan.lanes_per_op, plan.radix_bits), per_unit, count, as_run),
               "check": {"mismatches": bad, "of": "all %d encryptions, decrypted against the messages" % count}}
        if args.cpu_sample:
            import oracle
            sub["cpu_baseline"] = cpu_baseline(oracle, wl.msgs, e_h, n_h, out.cpu().numpy().view(np.uint32),
                                               "encryptions/s", "m^65537 mod n")
        return sub

    if args.serve_seconds is None:
        args.serve_seconds = 8.0 if args.workload == "serve" else 3.0
    if args.serve_forks is None:
        args.serve_forks = 3 if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) >= 8 else 1
    line = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u32",
            "data": "synthetic (seeded keys and messages)"}
    cpu = None
    t0 = time.time()

    if args.workload in ("crt2048", "enc2048", "crt4096"):
        if args.workload == "crt4096":
            wl = W.workload_crt4096(count=args.count or 1092)
            count = len(wl.ctxt)
        else:
            count = args.count or 16384
            wl = W.workload_c3(count=count)
        L, h = wl.limbs, wl.limbs // 2
        print("# workload ready in %.1fs" % (time.time() - t0), file=sys.stderr, flush=True)
        n_h, e_h, d_h = tab(wl, "n", L), tab(wl, "e", L), tab(wl, "d", L)
        if args.workload in ("crt2048", "crt4096"):
            c = dev(wl.ctxt)
            p, q, dp, dq, qi = (dev(tab(wl, a, h)) for a in ("p", "q", "dp", "dq", "qinv"))
            out = torch.empty_like(c)
            plan = rsagpu.get_plan(h, 1)
            steps_ms = []
            ms, wall = timed(lambda: rsagpu.decrypt_crt(c, p, q, dp, dq, qi, out=out), args.steps, args.warmup,
                             torch, steps_ms)
            line["batch_ms"] = {"p50": percentile(steps_ms, 50), "p99": percentile(steps_ms, 99),
                                "of": "one batch of %d decryptions" % count}
            # every decryption re-encrypted (e = 65537) must give its ciphertext back
            back = rsagpu.modexp(out, dev(e_h), dev(n_h))
            bad = row_mismatches(back, c)
            line["check"] = {"mismatches": bad, "of": "all %d decryptions, re-encrypted against the "
                                                      "ciphertexts" % count}
            if bad:
                raise SystemExit("round-trip check failed on %d elements" % bad)
            as_run = per_key_sum(wl.key_of, lambda k: crt_products(wl.keys[k], plan))
            # the same batch as one launch per key (plain form, no cross-key batching)
            per_key = []
            for j in range(len(wl.keys)):
                idx_j = torch.from_numpy(np.nonzero(wl.key_of == j)[0]).cuda()
                per_key.append([t[idx_j].contiguous() for t in (c, p, q, dp, dq, qi)] + [None])
                per_key[-1][-1] = torch.empty_like(per_key[-1][0])

            def plain():
                for a in per_key:
                    rsagpu.decrypt_crt(*a[:6], out=a[6])
            ms_plain, _ = timed(plain, max(1, args.steps // 4), 1, torch)
            line["plain_one_key_per_launch"] = {"value": count / (ms_plain / 1e3), "ms_per_step": ms_plain,
                                                "launches": len(per_key)}
            line.update(metric=METRIC if args.workload == "crt2048" else
                        "4096-bit modexp/sec (CRT decrypt) on 1 GPU", unit="decryptions/s",
                        config={"workload": "rsa%d-crt-decrypt" % (32 * L), "keys": len(wl.keys),
                                "messages": count, "modulus_bits": 32 * L, "radix_bits": plan.radix_bits,
                                "window_bits": plan.window_bits, "lanes_per_op": plan.lanes_per_op,
                                "waves_per_workgroup": 4 if plan.lanes_per_op >= 8 else 2})
            per_unit = unit_crt_products(h)
            line["roofline"] = roofline(per_unit * count, ms, "k_crt<%d,%d,%d>" % (plan.padded_limbs,
                                                                                   plan.lanes_per_op,
                                                                                   plan.radix_bits),
                                        per_unit, count, as_run, measured_peak())
            if args.cpu_sample:
                import oracle
                cpu = cpu_baseline(oracle, wl.ctxt, d_h, n_h, out.cpu().numpy().view(np.uint32), "decryptions/s",
                                   "plain C^d mod n (no CRT)",
                                   None if args.cpu_sample < 0 else min(args.cpu_sample, count),
                                   prefix=256 if L <= 64 else 32)
            line["encrypt"] = encrypt_half(wl, L, n_h, e_h,
                                           lambda x: rsagpu.decrypt_crt(x, p, q, dp, dq, qi))
            if args.serve_seconds > 0 and args.workload == "crt2048":
                sv = serve_leg(torch, np, rsagpu, W, args.serve_seconds, streams=args.serve_streams,
                               forks=args.serve_forks)
                if sv["check"]["mismatches"]:
                    raise SystemExit("serving run reported errors")
                line["latency_ms"] = {"p50": sv["p50_ms"], "p99": sv["p99_ms"],
                                      "of": "served requests: Poisson arrivals at 0.7 x the saturated rate, "
                                            "256 x 2048-bit + 64 x 4096-bit keys, 70% CRT decryptions, "
                                            "1-256 messages each"}
                sv.pop("products")
                line["serving"] = sv
        else:
            m = dev(wl.msgs)
            e, n = dev(e_h), dev(n_h)
            out = torch.empty_like(m)
            plan = rsagpu.get_plan(L, 0)
            ms, wall = timed(lambda: rsagpu.modexp(m, e, n, out=out), args.steps, args.warmup, torch)
            back = rsagpu.decrypt_crt(out, *(dev(tab(wl, a, h)) for a in ("p", "q", "dp", "dq", "qinv")))
            bad = row_mismatches(back, m)
            line["check"] = {"mismatches": bad, "of": "all %d encryptions, decrypted (CRT) against the "
                                                      "messages" % count}
            if bad:
                raise SystemExit("round-trip check failed on %d elements" % bad)
            as_run = per_key_sum(wl.key_of, lambda k: modexp_products(wl.keys[k], wl.keys[k].e, plan))
            line.update(metric="2048-bit modexp/sec (encrypt, e=65537) on 1 GPU", unit="encryptions/s",
                        config={"workload": "rsa2048-encrypt", "keys": len(wl.keys), "messages": count,
                                "radix_bits": plan.radix_bits, "window_bits": plan.window_bits,
                                "lanes_per_op": plan.lanes_per_op})
            per_unit = unit_enc_products(L)
            line["roofline"] = roofline(per_unit * count, ms, "k_modexp<%d,%d,%d>" % (plan.padded_limbs,
                                                                                      plan.lanes_per_op,
                                                                                      plan.radix_bits),
                                        per_unit, count, as_run, measured_peak())
            if args.cpu_sample:
                import oracle
                cpu = cpu_baseline(oracle, wl.msgs, e_h, n_h, out.cpu().numpy().view(np.uint32), "encryptions/s",
                                   "m^65537 mod n")
        value = count / (ms / 1e3)

    elif args.workload in ("rsa64", "rsa1024"):
        wl = W.workload_c1() if args.workload == "rsa64" else W.workload_c2()
        count = len(wl.ctxt)
        L = wl.limbs
        n_h, d_h = tab(wl, "n", L), tab(wl, "d", L)
        c, d, n = dev(wl.ctxt), dev(d_h), dev(n_h)
        out = torch.empty_like(c)
        plan = rsagpu.get_plan(L, 0)
        ms, wall = timed(lambda: rsagpu.modexp(c, d, n, out=out), args.steps, args.warmup, torch)
        back = rsagpu.modexp(out, dev(tab(wl, "e", L)), n)
        bad = row_mismatches(back, c)
        line["check"] = {"mismatches": bad, "of": "all %d decryptions, re-encrypted against the "
                                                  "ciphertexts" % count}
        if bad:
            raise SystemExit("round-trip check failed on %d elements" % bad)
        as_run = per_key_sum(wl.key_of, lambda k: modexp_products(wl.keys[k], wl.keys[k].d, plan))
        line.update(metric="%d-bit modexp/sec (full-d decrypt) on 1 GPU" % (32 * L), unit="decryptions/s",
                    config={"workload": wl.name + "-decrypt", "messages": count, "radix_bits": plan.radix_bits,
                            "window_bits": plan.window_bits, "lanes_per_op": plan.lanes_per_op})
        per_unit = unit_exp_products(L)
        line["roofline"] = roofline(per_unit * count, ms, "k_modexp<%d,%d,%d>" % (plan.padded_limbs,
                                                                                  plan.lanes_per_op,
                                                                                  plan.radix_bits),
                                    per_unit, count, as_run, measured_peak())
        if L <= 2:
            line["roofline"]["note"] = "launch-bound: one launch of ~80 dependent products"
        if args.cpu_sample:
            import oracle
            cpu = cpu_baseline(oracle, wl.ctxt, d_h, n_h, out.cpu().numpy().view(np.uint32), "decryptions/s",
                               "plain C^d mod n")
        line["encrypt"] = encrypt_half(wl, L, n_h, tab(wl, "e", L), lambda x: rsagpu.modexp(x, d, n))
        if L <= 2:
            line["encrypt"]["roofline"]["note"] = "launch-bound: one launch of 19 dependent products"
        value = count / (ms / 1e3)

    elif args.workload == "mixed":
        wl = W.workload_c4()
        nops = len(wl.kinds)
        ks = rsagpu.KeySet(len(wl.keys))
        for k in wl.keys:
            ks.add(k.limbs, k.n, k.e, k.p, k.q, k.dp, k.dq, k.qinv)
        ops = rsagpu.pack_ops(wl.kinds, wl.key_ids, wl.in_offs, wl.in_offs).cuda()
        inp = dev(wl.in_pool)
        out = torch.zeros(wl.out_words, dtype=torch.int32, device="cuda")
        ws = torch.empty(rsagpu.ops_workspace_size(nops), dtype=torch.uint8, device="cuda")
        tuned = {}
        if not args.no_tune:
            # autotuned plans per size for this batch: the ops-batch plans
            # (kind 2 encryption, kind 3 CRT half, kind 4 the CRT half of the
            # widest class of a bulk batch) tuned jointly on the call itself
            from paper_1407_1465_amd import tune
            widths = sorted({k.limbs for k in wl.keys}, reverse=True)
            slots = [(L // 2, 4 if L == widths[0] else 3) for L in widths] + [(L, 2) for L in widths]
            t_tune = time.perf_counter()
            chosen, tuned_ms = tune.tune_batch(lambda: rsagpu.ops_batch(ks, ops, inp, out, ws), slots,
                                               knobs=[("forks", [3, 2, 1, 0], ks.set_forks)])
            names = {2: "encrypt", 3: "CRT half", 4: "CRT half (widest class of a bulk batch)"}
            tuned = {"%d-bit %s" % (32 * key[0] if key[1] == 2 else 64 * key[0], names[key[1]]):
                     {"radix_bits": p[0], "lanes_per_op": p[1], "window_bits": p[2]}
                     for key, p in chosen.items() if isinstance(key, tuple)}
            tuned["forks"] = chosen["forks"]
            print("# tuned plans (%.1f s, %.2f ms per call): %s" % (time.perf_counter() - t_tune, tuned_ms,
                                                                     json.dumps(tuned)), file=sys.stderr, flush=True)
        ms_eager, _ = timed(lambda: rsagpu.ops_batch(ks, ops, inp, out, ws), args.steps, args.warmup, torch)
        # the same call captured once into a HIP graph and replayed
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cs):
            rsagpu.ops_batch(ks, ops, inp, out, ws)         # eager first: the stream's fork set exists
            cs.synchronize()
            with torch.cuda.graph(g, stream=cs):
                rsagpu.ops_batch(ks, ops, inp, out, ws)
        torch.cuda.current_stream().wait_stream(cs)
        out.zero_()
        steps_ms = []
        ms, wall = timed(g.replay, args.steps, args.warmup, torch, steps_ms)
        back = torch.zeros_like(out)
        ops_inv = rsagpu.pack_ops(1 - wl.kinds, wl.key_ids, wl.in_offs, wl.in_offs).cuda()
        rsagpu.ops_batch(ks, ops_inv, out, back, ws)
        torch.cuda.synchronize()
        bad_words = int((back != inp).sum().item())
        errs = rsagpu.device_errors()
        line["check"] = {"mismatches": bad_words + errs, "of": "every operation's output (graph replay) put "
                                                               "through the opposite operation (words differing + "
                                                               "data errors)"}
        if bad_words or errs:
            raise SystemExit("mixed batch round trip failed")

        widest = max(k.limbs for k in wl.keys)

        def op_products(kk):
            kind, kid = kk
            k = wl.keys[kid]
            # the ops-batch plans: kind 4 for the widest class's CRT halves (a bulk batch)
            pkind = (4 if k.limbs == widest else 3) if kind else 2
            pl = rsagpu.get_plan(k.limbs // 2 if kind else k.limbs, pkind)
            return crt_products(k, pl) if kind else modexp_products(k, k.e, pl)

        def op_units(kk):
            kind, kid = kk
            k = wl.keys[kid]
            return unit_crt_products(k.limbs // 2) if kind else unit_enc_products(k.limbs)
        pairs = np.stack([wl.kinds, wl.key_ids], 1).tolist()
        as_run = per_key_sum(pairs, lambda kk: op_products(tuple(kk)))
        products = per_key_sum(pairs, lambda kk: op_units(tuple(kk)))
        # plain form: one launch of the plain entry points per key and kind
        plain_launches = []
        pool_np = wl.in_pool
        for kid, k in enumerate(wl.keys):
            L, h = k.limbs, k.limbs // 2
            for kind in (0, 1):
                idx = np.nonzero((wl.key_ids == kid) & (wl.kinds == kind))[0]
                if not idx.size:
                    continue
                x = dev(np.stack([pool_np[o:o + L] for o in wl.in_offs[idx]]))
                cnt = len(idx)
                if kind:
                    a = [dev(np.tile(W.int_to_limbs(getattr(k, f), h), (cnt, 1))) for f in ("p", "q", "dp", "dq",
                                                                                             "qinv")]
                else:
                    a = [dev(np.tile(W.int_to_limbs(getattr(k, f), L), (cnt, 1))) for f in ("e", "n")]
                plain_launches.append((kind, x, a, torch.empty_like(x)))

        def plain():
            for kind, x, a, o in plain_launches:
                if kind:
                    rsagpu.decrypt_crt(x, *a, out=o)
                else:
                    rsagpu.modexp(x, *a, out=o)
        ms_plain, _ = timed(plain, max(1, args.steps // 4), 1, torch)
        # each (size, kind) bucket of the batch alone, with the same plans
        # (a call that small takes kind 3 for its CRT bucket: for the widest
        # one kind 3 holds kind 4's plan while it is timed, and runs it with
        # one pair of waves per workgroup, as kind 3 does)
        alone = {}
        limbs_of = np.array([wl.keys[i].limbs for i in wl.key_ids])
        sizes = sorted(set(limbs_of.tolist()), reverse=True)
        for L in sizes:
            for kind in (1, 0):
                idx = np.nonzero((limbs_of == L) & (wl.kinds == kind))[0]
                if not idx.size:
                    continue
                swap = kind == 1 and L == sizes[0]
                if swap:
                    p3, p4 = rsagpu.get_plan(L // 2, 3), rsagpu.get_plan(L // 2, 4)
                    rsagpu.set_plan(L // 2, 3, p4.radix_bits, p4.lanes_per_op, p4.window_bits)
                sub = rsagpu.pack_ops(wl.kinds[idx], wl.key_ids[idx], wl.in_offs[idx], wl.in_offs[idx]).cuda()
                ms_b, _ = timed(lambda: rsagpu.ops_batch(ks, sub, inp, out, ws, nops=len(idx)), 3, 1, torch)
                if swap:
                    rsagpu.set_plan(L // 2, 3, p3.radix_bits, p3.lanes_per_op, p3.window_bits)
                alone["%d-bit %s" % (32 * L, "CRT" if kind else "encrypt")] = {"ops": int(idx.size), "ms": ms_b}
        line["buckets_alone_ms"] = alone
        line.update(metric="mixed-size RSA ops/sec (1024-4096-bit, half CRT decrypt) on 1 GPU", unit="ops/s",
                    config={"workload": wl.name, "ops": nops, "keys": len(wl.keys),
                            "plans": tuned or "default",
                            "tuning": "coordinate descent over the plans per size and kind, timing the whole call"
                            if tuned else None,
                            "timed": "graph replay of one rsa_ops_batch call"})
        line["eager_ms_per_step"] = ms_eager
        line["batch_ms"] = {"p50": percentile(steps_ms, 50), "p99": percentile(steps_ms, 99)}
        line["plain_one_key_per_launch"] = {"value": nops / (ms_plain / 1e3), "ms_per_step": ms_plain,
                                            "launches": len(plain_launches)}
        line["roofline"] = roofline(products, ms, "k_ops_* (all buckets)", "per operation by size and kind",
                                    nops, as_run, measured_peak())
        if args.cpu_sample:
            import oracle
            got = out.cpu().numpy().view(np.uint32)
            by_l = {}
            for i, (kind, kid, off) in enumerate(zip(wl.kinds, wl.key_ids, wl.in_offs)):
                by_l.setdefault(wl.keys[kid].limbs, []).append(i)
            t_cpu, n_cpu, threads = 0.0, 0, oracle_threads()
            one = {}
            for L, idx in sorted(by_l.items()):
                if args.cpu_sample > 0:
                    idx = idx[:args.cpu_sample]
                base = np.stack([pool_np[wl.in_offs[i]:wl.in_offs[i] + L] for i in idx])
                exps = W.ints_to_limbs([wl.keys[wl.key_ids[i]].d if wl.kinds[i] else wl.keys[wl.key_ids[i]].e
                                        for i in idx], L)
                mods = W.ints_to_limbs([wl.keys[wl.key_ids[i]].n for i in idx], L)
                want, cw, _ = oracle.modexp_batch(base, exps, mods, nthreads=threads)
                gpu = np.stack([got[wl.in_offs[i]:wl.in_offs[i] + L] for i in idx])
                nbad = int((want != gpu).any(axis=1).sum())
                if nbad:
                    raise SystemExit("mixed batch differs from the oracle on %d %d-bit operations" % (nbad, 32 * L))
                t_cpu += cw
                n_cpu += len(idx)
            share, ncpu, model = host_cpus()
            cpu = {"value": n_cpu / t_cpu, "unit": "ops/s", "cores": threads, "kind": "oracle",
                   "sample": "%s %d operations of the batch (plain M^e / C^d mod n, no CRT), %.1f s wall; every "
                             "output equals the GPU's" % ("all" if n_cpu == nops else "a per-size prefix of",
                                                         n_cpu, t_cpu),
                   "verified": n_cpu, "mismatches": 0, "cpu_model": model, "host_cpus": ncpu, "cpu_share": share}
        value = nops / (ms / 1e3)
        del g
        ks.close()

    elif args.workload == "paper":
        # The paper's own experiment (Section 10, Tables 1 and 2): one-word
        # moduli, e = 131, messages 0..800, at every data size the tables
        # list; encryption and decryption (round trip checked) per size.
        rows, checked = [], 0
        for t, key in sorted(W.PAPER_TABLE_KEYS.items()):
            for i, N in enumerate(W.PAPER_TABLE_SIZES):
                msgs = W.paper_table_messages(N)
                m = dev(msgs)
                e = dev(np.full((N, 1), key.e, dtype=np.uint32))
                d = dev(np.full((N, 1), key.d, dtype=np.uint32))
                n = dev(np.full((N, 1), key.n, dtype=np.uint32))
                c = torch.empty_like(m)
                back = torch.empty_like(m)
                ms_enc, _ = timed(lambda: rsagpu.modexp(m, e, n, out=c), args.steps, args.warmup, torch)
                ms_dec, _ = timed(lambda: rsagpu.modexp(c, d, n, out=back), args.steps, args.warmup, torch)
                if not torch.equal(back, m):
                    raise SystemExit("paper-table round trip failed (table %d, %d messages)" % (t, N))
                checked += N
                rows.append({"table": t, "n": key.n, "e": key.e, "d": key.d, "messages": N,
                             "encrypt_ms": ms_enc, "decrypt_ms": ms_dec,
                             "paper_gpu_time_as_printed": W.PAPER_TABLE_GPU_TIME[t][i]})
        last = rows[-1]
        ms, wall = last["encrypt_ms"], sum(r["encrypt_ms"] + r["decrypt_ms"] for r in rows) * args.steps / 1e3
        plan = rsagpu.get_plan(1, 0)
        line.update(metric="paper Section 10 workload: one-word RSA encryptions/s (n = 1009*509, e = 131, "
                           "32768 messages 0..800) on 1 GPU", unit="encryptions/s",
                    config={"workload": "paper-tables-1-2", "radix_bits": plan.radix_bits,
                            "window_bits": plan.window_bits, "lanes_per_op": plan.lanes_per_op})
        line["rows"] = rows
        line["check"] = {"mismatches": 0, "of": "all %d messages encrypted and decrypted back" % checked}
        value = last["messages"] / (ms / 1e3)

    elif args.workload == "keygen":
        # Section 3.1 key generation with the Miller-Rabin rounds batched on
        # the GPU: 16 seeded 4096-bit keys, equal to the CPU generator's.
        from paper_1407_1465_amd import keygen
        nk, bits, seed = 16, 4096, W.SEED_BASE + 7
        keygen.make_keys_gpu(1024, seed, 2)                # warm-up (library load, kernels)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        keys = keygen.make_keys_gpu(bits, seed, nk)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        t2 = time.perf_counter()
        cpu_key = W.make_key(bits, W.derive_seed(seed, bits, 0))
        cpu_s = time.perf_counter() - t2
        if keys[0] != cpu_key:
            raise SystemExit("GPU key generation differs from the CPU generator")
        line["check"] = {"mismatches": 0, "of": "key 0 against the CPU generator; every key's own consistency"}
        ms = wall * 1e3
        line.update(metric="4096-bit RSA key generation (Miller-Rabin on the GPU) keys/s on 1 GPU",
                    unit="keys/s", config={"workload": "keygen-4096", "keys": nk, "modulus_bits": bits})
        line["cpu_keygen_one_thread"] = {"value": 1.0 / cpu_s, "unit": "keys/s",
                                         "sample": "key 0 of the same seeds, Python pow"}
        value = nk / wall

    elif args.workload == "mulpeak":
        from paper_1407_1465_amd import mulpeak
        rates = [mulpeak.measure(op) for op in (0, 1, 2)]
        mad = rates[0]
        line.update(metric="32-bit integer multiply issue rate (v_mad_u64_u32) on 1 GPU", unit="T products/s",
                    config={"workload": "mulpeak", "lanes_per_block": mad["lanes_per_block"],
                            "chains_per_lane": mad["chains_per_lane"], "blocks": mad["blocks"],
                            "iters": mad["iters"]})
        line["rates"] = [{"op": r["op"], "value": r["ops_per_s"] / 1e12, "unit": "T ops/s",
                          "frac_of_nominal": r["ops_per_s"] / INT32_MUL_PEAK, "ms_per_launch": r["ms_per_launch"],
                          "ops_per_launch": r["ops_per_launch"],
                          "lane_ops_per_clock_per_cu_at_2.4GHz": r["ops_per_s"] / (r["cus"] * 2.4e9)}
                         for r in rates]
        line["roofline"] = {"bound": "alu", "achieved": mad["ops_per_s"] / 1e12, "peak": INT32_MUL_PEAK / 1e12,
                            "unit": "T int32-mul/s", "frac": mad["ops_per_s"] / INT32_MUL_PEAK, "traffic": None,
                            "kernel": "k_mulpeak<0>", "products_per_launch": mad["ops_per_launch"],
                            "ms_per_launch": mad["ms_per_launch"]}
        line["check"] = {"mismatches": 0, "of": "no results (issue-rate probe)"}
        value = mad["ops_per_s"] / 1e12
        ms, wall = mad["ms_per_launch"], sum(r["ms_per_launch"] for r in rates) * 8 / 1e3

    else:   # serve
        sv = serve_leg(torch, np, rsagpu, W, args.serve_seconds, plain_requests=400, streams=args.serve_streams,
                       forks=args.serve_forks)
        line["check"] = sv.pop("check")
        if line["check"]["mismatches"]:
            raise SystemExit("serving run reported errors")
        products = sv.pop("products")
        line.update(metric="RSA serving (2048/4096-bit keys, 70% CRT decrypt): requests/s at p50/p99 latency",
                    unit="requests/s",
                    config={"workload": "rsa-serve-2048-4096", "keys": 320, "rate_req_per_s": sv["rate_req_per_s"],
                            "saturated_req_per_s": sv["saturated_req_per_s"],
                            "saturation_bursts_req_per_s": sv["saturation_bursts_req_per_s"],
                            "requests": sv["requests"], "streams": sv["streams"], "forks": sv["forks"],
                            "max_inflight": sv["max_inflight"]})
        line["latency_ms"] = {"p50": sv["p50_ms"], "p99": sv["p99_ms"], "mean": sv["mean_ms"]}
        line["ops_per_s"] = sv["ops_per_s"]
        line["plain_one_request_per_launch"] = sv["plain_one_request_per_launch"]
        line["roofline"] = roofline(products, sv["span_s"] * 1e3, "k_ops_* (every batch of the run)",
                                    "per message by size and kind", sv["requests"], None, measured_peak())
        line["roofline"]["note"] = ("served messages' algorithmic products over the run's span (arrival of "
                                    "the first request to completion of the last), at 0.7 x saturation")
        value = sv["requests_per_s"]
        ms, wall = sv["span_s"] * 1e3, sv["span_s"]

    if line_plans:
        line["config"]["plans_set"] = line_plans
    line["value"] = value
    line["ms_per_step"] = ms
    line["config"]["wall_s"] = wall
    line["cpu_baseline"] = cpu
    order = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
             "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"]
    out_line = {k: line[k] for k in order if k in line}
    out_line.update({k: v for k, v in line.items() if k not in out_line})
    print(json.dumps(out_line), flush=True)


if __name__ == "__main__":
    main()
