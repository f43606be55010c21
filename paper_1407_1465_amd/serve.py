"""Continuous-batching request loop over resident keys.

A request is one key and one kind (encrypt with e, or CRT decrypt) applied to
1..256 messages.  The server keeps the keys and their Montgomery constants
resident (a keyset), and runs a scheduler tick loop:

  1. retire batches whose completion event has fired: their outputs are
     already in pinned host memory; free their pool slots, finish requests;
  2. admit waiting requests in arrival order while their messages fit the
     device pool (memory-based admission: the input and output slots a
     request needs are reserved from a fixed budget; the first request that
     does not fit blocks the ones behind it, so admission is FIFO-fair);
  3. while fewer than `max_inflight` batches are on the GPU, pack every
     admitted request into one batch of operation descriptors and launch it
     on an idle stream (one host-to-device copy of the descriptors and one of
     the packed inputs, one rsa_ops_batch call, one device-to-host copy of
     the outputs, an event).

Requests that arrive while others are on the GPU are admitted as slots free
up and launched in the next batch, so their work overlaps the running batch
on the device.  Results do not depend on batching: each operation's output
is a function of its key and input only.

The executor is pluggable: `GpuExecutor` drives the library; tests use a CPU
stand-in with the same interface to check the scheduling logic.
"""
from __future__ import annotations

import heapq
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclass
class Request:
    rid: int
    key_id: int
    kind: int                   # 0 encrypt, 1 CRT decrypt
    inputs: np.ndarray          # (count, limbs) uint32
    arrival: float = 0.0        # seconds on the server clock
    done: float = -1.0
    outputs: Optional[np.ndarray] = None
    error: Optional[str] = None
    # filled by the scheduler
    in_off: int = -1
    out_off: int = -1

    @property
    def words(self) -> int:
        return int(self.inputs.size)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class SlotPool:
    """First-fit allocator of word ranges inside a fixed pool."""

    def __init__(self, words: int):
        self.words = words
        self.free: List[List[int]] = [[0, words]]        # sorted [start, length]
        self.used = 0

    def alloc(self, n: int) -> int:
        for i, (start, length) in enumerate(self.free):
            if length >= n:
                if length == n:
                    self.free.pop(i)
                else:
                    self.free[i] = [start + n, length - n]
                self.used += n
                return start
        return -1

    def release(self, start: int, n: int) -> None:
        self.used -= n
        self.free.append([start, n])
        self.free.sort()
        merged: List[List[int]] = []
        for s, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1][1] += l
            else:
                merged.append([s, l])
        self.free = merged


@dataclass
class Batch:
    requests: List[Request]
    handle: object = None
    launched: float = 0.0


class Server:
    """Scheduler of requests onto an executor (see module docstring)."""

    def __init__(self, executor, pool_words: int, max_inflight: int = 2, max_ops: int = 65536,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.in_pool = SlotPool(pool_words)
        self.out_pool = SlotPool(pool_words)
        self.max_inflight = max_inflight
        self.max_ops = max_ops
        self.clock = clock
        self.t0 = clock()
        self.waiting: List[Request] = []       # FIFO
        self.admitted: List[Request] = []
        self.inflight: List[Batch] = []
        self.finished: List[Request] = []
        self.rejected: List[Request] = []

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request) -> None:
        if req.words > self.in_pool.words or len(req.inputs) > self.max_ops:
            req.error = "request larger than the device pool"
            req.done = self.now()
            self.rejected.append(req)
            return
        self.waiting.append(req)

    def _retire(self) -> None:
        still = []
        for b in self.inflight:
            if self.ex.poll(b.handle):
                try:
                    outs = self.ex.collect(b.handle)
                    err = None
                except Exception as e:                       # executor failure: this batch only
                    outs, err = None, str(e)
                t = self.now()
                for r in b.requests:
                    if err is None:
                        r.outputs = outs[r.rid]
                    else:
                        r.error = err
                    r.done = t
                    self.in_pool.release(r.in_off, r.words)
                    self.out_pool.release(r.out_off, r.words)
                    self.finished.append(r)
            else:
                still.append(b)
        self.inflight = still

    def _admit(self) -> None:
        while self.waiting:
            r = self.waiting[0]
            a = self.in_pool.alloc(r.words)
            if a < 0:
                return
            b = self.out_pool.alloc(r.words)
            if b < 0:
                self.in_pool.release(a, r.words)
                return
            r.in_off, r.out_off = a, b
            self.admitted.append(self.waiting.pop(0))

    def _launch(self) -> None:
        while self.admitted and len(self.inflight) < self.max_inflight:
            batch, nops = [], 0
            while self.admitted and nops + len(self.admitted[0].inputs) <= self.max_ops:
                r = self.admitted.pop(0)
                batch.append(r)
                nops += len(r.inputs)
            if not batch:
                return
            b = Batch(batch, launched=self.now())
            b.handle = self.ex.launch(batch)
            self.inflight.append(b)

    def tick(self) -> None:
        self._retire()
        self._admit()
        self._launch()

    def idle(self) -> bool:
        return not (self.waiting or self.admitted or self.inflight)

    def run(self, arrivals: Sequence[Request], poll_sleep: float = 0.0) -> None:
        """Open-loop run: request i is submitted once the clock passes its
        arrival time; returns when every request has finished."""
        pending = sorted(arrivals, key=lambda r: r.arrival)
        i = 0
        self.t0 = self.clock()
        while i < len(pending) or not self.idle():
            t = self.now()
            while i < len(pending) and pending[i].arrival <= t:
                self.submit(pending[i])
                i += 1
            self.tick()
            if poll_sleep:
                time.sleep(poll_sleep)

    def stats(self) -> Dict[str, float]:
        done = [r for r in self.finished if r.error is None]
        lat = np.array([r.latency for r in done]) if done else np.zeros(1)
        span = max((r.done for r in self.finished), default=0.0) - min((r.arrival for r in self.finished),
                                                                        default=0.0)
        ops = sum(len(r.inputs) for r in done)
        return {
            "requests": len(done),
            "errors": sum(1 for r in self.finished if r.error is not None),
            "rejected": len(self.rejected),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "requests_per_s": len(done) / span if span > 0 else 0.0,
            "ops_per_s": ops / span if span > 0 else 0.0,
            "span_s": span,
        }


class GpuExecutor:
    """Runs batches through rsa_ops_batch, each on an idle stream of its own
    (at most one uncollected batch per stream, so max_inflight = streams).

    A batch's inputs are packed back to back into the stream's pinned host
    staging buffer and go to the device in one copy; its outputs come back
    in one copy into the stream's pinned output buffer, from which collect()
    slices each request.  The server's slot pools bound the words in flight
    (memory-based admission); every stream's staging holds a full pool."""

    def __init__(self, keyset, limbs_of_key: Sequence[int], pool_words: int, max_ops: int,
                 streams: int = 2, forks: Optional[int] = None):
        import torch
        from . import rsagpu
        self.torch = torch
        self.rsagpu = rsagpu
        self.ks = keyset
        if forks is not None:
            # streams a batch forks its widest CRT buckets onto, per executor
            # stream: streams x (forks + 1) streams, which overlap only while
            # the runtime has a hardware queue for each (GPU_MAX_HW_QUEUES,
            # 4 by default, one of them the null stream's)
            keyset.set_forks(forks)
        self.forks = forks
        self.limbs = np.asarray(list(limbs_of_key), dtype=np.int64)
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.in_dev = [torch.zeros(pool_words, dtype=torch.int32, device="cuda") for _ in range(streams)]
        self.out_dev = [torch.zeros(pool_words, dtype=torch.int32, device="cuda") for _ in range(streams)]
        self.in_host = [torch.zeros(pool_words, dtype=torch.int32, pin_memory=True) for _ in range(streams)]
        self.out_host = [torch.zeros(pool_words, dtype=torch.int32, pin_memory=True) for _ in range(streams)]
        self.in_np = [t.numpy().view(np.uint32) for t in self.in_host]
        self.out_np = [t.numpy().view(np.uint32) for t in self.out_host]
        wsb = rsagpu.ops_workspace_size(max_ops)
        self.ws = [torch.empty(wsb, dtype=torch.uint8, device="cuda") for _ in range(streams)]
        self.ops_host = [torch.zeros((max_ops, 3), dtype=torch.int64, pin_memory=True) for _ in range(streams)]
        self.ops_np = [t.numpy() for t in self.ops_host]
        self.ops_dev = [torch.zeros((max_ops, 3), dtype=torch.int64, device="cuda") for _ in range(streams)]
        self.pool_words = pool_words
        self.max_ops = max_ops
        self.max_inflight = streams
        self.busy = [False] * streams           # a launched batch not yet collected

    def _idle_stream(self) -> int:
        for k, b in enumerate(self.busy):
            if not b:
                return k
        raise RuntimeError("every stream has a batch in flight (more batches than streams)")

    def launch(self, reqs: List[Request]):
        torch = self.torch
        k = self._idle_stream()
        s = self.streams[k]
        counts = np.fromiter((len(r.inputs) for r in reqs), dtype=np.int64, count=len(reqs))
        kinds = np.fromiter((r.kind for r in reqs), dtype=np.int64, count=len(reqs))
        kids = np.fromiter((r.key_id for r in reqs), dtype=np.int64, count=len(reqs))
        nops = int(counts.sum())
        if nops > self.max_ops:
            raise ValueError("batch of %d operations exceeds max_ops" % nops)
        op_words = np.repeat(self.limbs[kids], counts)
        offs = np.zeros(nops, dtype=np.int64)
        np.cumsum(op_words[:-1], out=offs[1:])
        total = int(offs[-1] + op_words[-1]) if nops else 0
        if total > self.pool_words:
            raise ValueError("batch of %d words exceeds the staging buffers" % total)
        ops = self.ops_np[k]
        ops[:nops, 0] = np.repeat(kinds, counts) | (np.repeat(kids, counts) << 32)
        ops[:nops, 1] = offs
        ops[:nops, 2] = offs
        if reqs:
            np.concatenate([r.inputs.reshape(-1) for r in reqs], out=self.in_np[k][:total])
        first = np.zeros(len(reqs), dtype=np.int64)
        np.cumsum(counts[:-1], out=first[1:])
        with torch.cuda.stream(s):
            self.ops_dev[k][:nops].copy_(self.ops_host[k][:nops], non_blocking=True)
            self.in_dev[k][:total].copy_(self.in_host[k][:total], non_blocking=True)
            self.rsagpu.ops_batch(self.ks, self.ops_dev[k], self.in_dev[k], self.out_dev[k], self.ws[k], nops=nops,
                                  stream=s)
            self.out_host[k][:total].copy_(self.out_dev[k][:total], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self.busy[k] = True
        starts = offs[first] if nops else first
        return (ev, reqs, k, starts)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def collect(self, handle):
        ev, reqs, k, starts = handle
        ev.synchronize()
        out = self.out_np[k]
        res = {r.rid: out[o:o + r.words].reshape(r.inputs.shape).copy() for r, o in zip(reqs, starts.tolist())}
        self.busy[k] = False
        return res


def poisson_requests(rate: float, n: int, seed: int, key_limbs: Sequence[int], key_moduli: Sequence[int],
                     decrypt_frac: float = 0.7, max_msgs: int = 256,
                     key_weights: Optional[Sequence[float]] = None) -> List[Request]:
    """n requests with exponential inter-arrival times (rate per second); each
    picks a key (uniformly unless weighted), a kind (decrypt with probability
    decrypt_frac) and 1..max_msgs messages uniform in [0, n)."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    nk = len(key_limbs)
    w = None if key_weights is None else np.asarray(key_weights, dtype=float) / np.sum(key_weights)
    for i in range(n):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        kid = int(rng.choice(nk, p=w))
        kind = int(rng.random() < decrypt_frac)
        cnt = int(rng.integers(1, max_msgs + 1))
        msgs = W.uniform_below(key_moduli[kid], cnt, W.derive_seed(seed, i, 5), key_limbs[kid])
        out.append(Request(i, kid, kind, msgs, arrival=t))
    return out
