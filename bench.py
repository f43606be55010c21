#!/usr/bin/env python3
"""Benchmark: batched RSA modular exponentiation on one MI355X.

Default workload: 2048-bit RSA, 64 seeded keys, 16384 messages assigned
round-robin, CRT decryption (two 1024-bit exponentiations with dp, dq and
Garner recombination per message).  One step = one CRT-decryption pass over
the whole batch, inputs resident in HBM.  The line printed is

  {"metric", "value" (decryptions/s), ..., "roofline": {...}, "cpu_baseline": {...}}

`roofline` rates the decryption kernel against the chip's 32-bit integer
multiply peak: algorithmic 32x32-bit products per launch (Montgomery products
of the fixed-window method, 2h^2 + h products each, plus the recombination)
divided by the kernel's mean launch time from HIP events on its stream.
`cpu_baseline` times the plain CPU oracle (C^d mod n, no CRT) on a bounded
sample of the same messages on the host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 256 CUs x 64 lanes x 2.4 GHz / 4: the 32x32->64-bit integer multiply
# (v_mad_u64_u32) issues at a quarter of the full VALU rate.
INT32_MUL_PEAK = 256 * 64 * 2.4e9 / 4
METRIC = "2048-bit modexp/sec (CRT decrypt) on 1 GPU, %INT32-mul peak; p50/p99 latency"


def fixed_window_montmuls(ebits: int, w: int) -> int:
    """Montgomery products of the fixed-window method for an ebits-bit
    exponent: (ceil(b/w) - 1)(w + 1) + 2^w."""
    nwin = -(-ebits // w)
    return (nwin - 1) * (w + 1) + (1 << w)


def crt_products(key, plan_w: int) -> int:
    h = key.limbs // 2
    per_mont = 2 * h * h + h
    mm = fixed_window_montmuls(key.dp.bit_length(), plan_w) + \
        fixed_window_montmuls(key.dq.bit_length(), plan_w)
    return mm * per_mont + (2 * h * h + h) + h * h


def modexp_products(key, ebits: int, plan_w: int) -> int:
    s = key.limbs
    return fixed_window_montmuls(ebits, plan_w) * (2 * s * s + s)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--count", type=int, default=16384)
    ap.add_argument("--keys", type=int, default=64)
    ap.add_argument("--cpu-sample", type=int, default=512,
                    help="messages the CPU oracle decrypts for the baseline (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(operations are independent; see the sharding note in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1407_1465_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build()
    from paper_1407_1465_amd import rsagpu
    from paper_1407_1465_amd import workloads as W

    t0 = time.time()
    wl = W.workload_c3(count=args.count, nkeys=args.keys)
    L = wl.limbs
    h = L // 2
    print("# workload ready in %.1fs: %d keys, %d messages, %d-bit" %
          (time.time() - t0, len(wl.keys), args.count, 32 * L), file=sys.stderr, flush=True)

    def tab(attr, width):
        return np.ascontiguousarray(
            W.ints_to_limbs([getattr(k, attr) for k in wl.keys], width)[wl.key_of])

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()

    torch.cuda.set_device(0)
    c = dev(wl.ctxt)
    p, q, dp, dq, qi = (dev(tab(a, h)) for a in ("p", "q", "dp", "dq", "qinv"))
    out = torch.empty_like(c)
    plan = rsagpu.get_plan(h, 1)

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        rsagpu.decrypt_crt(c, p, q, dp, dq, qi, out=out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        rsagpu.decrypt_crt(c, p, q, dp, dq, qi, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    value = args.count / (ms_per_step / 1e3)
    if rsagpu.device_errors() != 0:
        raise SystemExit("device reported data errors")

    # spot-check a few outputs against the round trip before reporting
    e_full = dev(tab("e", L))
    n_full = dev(tab("n", L))
    idx = torch.arange(0, args.count, max(1, args.count // 64), device="cuda")
    back = rsagpu.modexp(out[idx].contiguous(), e_full[idx].contiguous(), n_full[idx].contiguous())
    if not torch.equal(back, c[idx]):
        raise SystemExit("round-trip check failed")

    products = sum(crt_products(wl.keys[k], plan.window_bits) for k in wl.key_of.tolist())
    achieved = products / (ms_per_step / 1e3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_MUL_PEAK / 1e12,
                "unit": "T int32-mul/s", "frac": achieved / INT32_MUL_PEAK, "traffic": None,
                "kernel": "k_crt<32,%d>" % plan.lanes_per_op,
                "products_per_launch": products}

    cpu = None
    if args.cpu_sample > 0:
        import oracle
        ns = min(args.cpu_sample, args.count)
        n_h = tab("n", L)[:ns]
        d_h = tab("d", L)[:ns]
        threads = min(16, os.cpu_count() or 1)
        got, cwall, used = oracle.modexp_batch(wl.ctxt[:ns], d_h, n_h, nthreads=threads)
        gpu_h = out[:ns].cpu().numpy().view(np.uint32)
        if not np.array_equal(got, gpu_h):
            raise SystemExit("GPU output differs from the oracle on the CPU sample")
        cpu = {"value": ns / cwall, "unit": "decryptions/s", "cores": used, "kind": "oracle",
               "sample": "first %d messages of the same batch, plain C^d mod n (no CRT), "
                         "%.1f s wall" % (ns, cwall)}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "decryptions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded keys and messages)",
        "config": {"workload": "rsa2048-crt-decrypt", "keys": len(wl.keys), "messages": args.count,
                   "modulus_bits": 32 * L, "window_bits": plan.window_bits,
                   "lanes_per_op": plan.lanes_per_op, "wall_s": wall},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
