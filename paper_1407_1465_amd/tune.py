"""Autotuned plans, cached on disk per device architecture.

`tune(limbs, kind, exp_bits, count)` runs the library's autotuner
(rsa_autotune: every compiled kernel instance of the width class at every
window that fits, timed on synthetic operands of the given batch size: plain
calls for kinds 0 and 1, rsa_ops_batch on a synthetic keyset for kinds 2 to
4) and records the winner in a JSON cache; `apply_cached()` re-installs
cached plans with rsa_set_plan so later processes skip the search.  Entries
are keyed by the GPU architecture, the operand width in words, the kind, the
exponent length and the batch size rounded up to a power of two.

`tune_batch(run, slots)` tunes the plans of a whole rsa_ops_batch call
jointly: the buckets of a mixed batch run side by side and compete for the
CUs (registers, LDS, issue slots), so the plan that is fastest for a bucket
alone (often the one with the shortest chain) need not be the fastest in the
mix.  It installs each candidate plan of one (width, kind) slot at a time
and times the real call, keeping the fastest (coordinate descent).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

import torch

from . import rsagpu

_DEFAULT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".tunecache",
                        "plans.json")


def cache_path() -> str:
    return os.environ.get("RSAGPU_TUNE_FILE", _DEFAULT)


def _arch() -> str:
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


CRT_KINDS = (1, 3, 4)


def plan_width(limbs: int, kind: int) -> int:
    """Width whose class a plan of `kind` is stored under (CRT: one half)."""
    return limbs // 2 if kind in CRT_KINDS else limbs


def _key(limbs: int, kind: int, exp_bits: int, count: int) -> str:
    bucket = 1 << max(0, (count - 1).bit_length())
    return "%s/w%d/k%d/e%d/n%d" % (_arch(), limbs, kind, exp_bits, bucket)


def load() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(cache: Dict[str, dict]) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(limbs: int, kind: int, exp_bits: int, count: int, use_cache: bool = True) -> rsagpu.Plan:
    """Best plan for (limbs, kind, exp_bits, count), installed in the library."""
    cache = load()
    key = _key(limbs, kind, exp_bits, count)
    width = plan_width(limbs, kind)
    if use_cache and key in cache:
        e = cache[key]
        rsagpu.set_plan(width, kind, e["radix_bits"], e["lanes_per_op"], e["window_bits"])
        return rsagpu.get_plan(width, kind)
    plan = rsagpu.autotune(limbs, kind, exp_bits, count)
    cache[key] = {"radix_bits": plan.radix_bits, "lanes_per_op": plan.lanes_per_op,
                  "window_bits": plan.window_bits, "padded_limbs": plan.padded_limbs}
    save(cache)
    return plan


def apply_cached(arch: Optional[str] = None) -> int:
    """Installs every cached plan of this architecture; returns how many."""
    arch = arch or _arch()
    n = 0
    for key, e in load().items():
        parts = key.split("/")
        if parts[0] != arch:
            continue
        limbs, kind = int(parts[1][1:]), int(parts[2][1:])
        width = plan_width(limbs, kind)
        rsagpu.set_plan(width, kind, e["radix_bits"], e["lanes_per_op"], e["window_bits"])
        n += 1
    return n


def candidate_plans(width: int, kind: int):
    """(radix_bits, lanes_per_op, window_bits) the library accepts for the
    width class of `width` and plan `kind` (the current plan is restored;
    none where the class has no plan of that kind)."""
    try:
        cur = rsagpu.get_plan(width, kind)
    except rsagpu.RSAError:
        return []
    out = []
    for radix in (32, 29):
        for lanes in (1, 2, 4, 8, 16):
            for w in range(2, 7):
                try:
                    rsagpu.set_plan(width, kind, radix, lanes, w)
                except rsagpu.RSAError:
                    continue
                out.append((radix, lanes, w))
    rsagpu.set_plan(width, kind, cur.radix_bits, cur.lanes_per_op, cur.window_bits)
    return out


def tune_batch(run, slots, reps: int = 3, passes: int = 1, tolerance: float = 0.005, knobs=(),
               timer=None, confirm: int = 5):
    """Coordinate descent over the plans of `slots` [(width, kind), ...] for
    the batch that run() enqueues on torch's current stream: each candidate
    is installed and the batch timed (one warm-up, then `reps` runs between
    HIP events); a candidate replaces the slot's plan when it is faster by
    more than `tolerance` in two timings in a row (one lucky timing does not
    move the descent).  `knobs` [(name, values, apply)] are further settings
    tuned the same way after the plans (apply(value) installs one; values[0]
    is the current one).  At the end the starting settings and the chosen
    ones are timed `confirm` times each, alternately, and the chosen ones are
    kept only if their median is faster by more than `tolerance`; otherwise
    the starting settings are restored.  `timer`, if given, replaces the HIP
    event timing (a callable returning ms per call).  Returns ({(width,
    kind): (radix, lanes, window), name: value, ...}, ms per call with the
    settings in place)."""
    if timer is None:
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

        def timer() -> float:
            run()
            e0.record(stream)
            for _ in range(reps):
                run()
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / reps

    def plan_of(width, kind):
        p = rsagpu.get_plan(width, kind)
        return (p.radix_bits, p.lanes_per_op, p.window_bits)

    def install(cfg):
        for key, value in cfg.items():
            if isinstance(key, tuple):
                rsagpu.set_plan(key[0], key[1], *value)
        for name, _, apply in knobs:
            apply(cfg[name])

    start = {(w, k): plan_of(w, k) for w, k in slots}
    for name, values, _ in knobs:
        start[name] = values[0]

    def better(ms, best):
        return ms < best * (1.0 - tolerance)

    best = timer()
    chosen = dict(start)
    for _ in range(passes):
        for width, kind in slots:
            cur = chosen[(width, kind)]
            for cand in candidate_plans(width, kind):
                if cand == cur:
                    continue
                rsagpu.set_plan(width, kind, *cand)
                ms = timer()
                if better(ms, best):
                    ms2 = timer()
                    if better(ms2, best):
                        best, cur = max(ms, ms2), cand
            rsagpu.set_plan(width, kind, *cur)
            chosen[(width, kind)] = cur
        for name, values, apply in knobs:
            cur = chosen[name]
            for v in values:
                if v == cur:
                    continue
                apply(v)
                ms = timer()
                if better(ms, best):
                    ms2 = timer()
                    if better(ms2, best):
                        best, cur = max(ms, ms2), v
            apply(cur)
            chosen[name] = cur
    if chosen == start:
        return chosen, best
    a, b = [], []
    for _ in range(confirm):
        install(start)
        a.append(timer())
        install(chosen)
        b.append(timer())
    a.sort()
    b.sort()
    if better(b[len(b) // 2], a[len(a) // 2]):
        return chosen, b[len(b) // 2]
    install(start)
    return dict(start), a[len(a) // 2]
