"""Scheduling logic of the continuous-batching server, on the CPU with a
stand-in executor and a fake clock (no GPU)."""
import numpy as np
import pytest

from paper_1407_1465_amd import workloads as W
from paper_1407_1465_amd.serve import Request, Server, SlotPool, poisson_requests


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Completes a batch `delay` fake seconds after launch; computes results
    with Python integers; can be told to fail a given batch."""

    def __init__(self, clock, keys, delay=1.0, fail_batches=()):
        self.clock, self.keys, self.delay = clock, keys, delay
        self.launched = []
        self.fail = set(fail_batches)

    def launch(self, reqs):
        self.launched.append([r.rid for r in reqs])
        return (len(self.launched) - 1, self.clock() + self.delay, reqs)

    def poll(self, h):
        return self.clock() >= h[1]

    def collect(self, h):
        idx, _, reqs = h
        if idx in self.fail:
            raise RuntimeError("device failure in batch %d" % idx)
        out = {}
        for r in reqs:
            k = self.keys[r.key_id]
            x = r.kind and k.d or k.e
            vals = [pow(v, x, k.n) for v in W.limbs_to_ints(r.inputs)]
            out[r.rid] = W.ints_to_limbs(vals, k.limbs)
        return out


def drive(server, clock, reqs, step=0.25, limit=10000):
    pending = sorted(reqs, key=lambda r: r.arrival)
    i = 0
    for _ in range(limit):
        while i < len(pending) and pending[i].arrival <= clock.t:
            server.submit(pending[i])
            i += 1
        server.tick()
        if i == len(pending) and server.idle():
            return
        clock.t += step
    raise AssertionError("server did not drain")


@pytest.fixture(scope="module")
def keys():
    return W.make_keys(128, 31, 3)


def mk(keys, rid, kid, kind, count, arrival, seed=0):
    k = keys[kid]
    msgs = W.uniform_below(k.n, count, seed * 1000 + rid, k.limbs)
    return Request(rid, kid, kind, msgs, arrival=arrival)


def test_slot_pool_first_fit_and_merge():
    p = SlotPool(100)
    a, b, c = p.alloc(30), p.alloc(30), p.alloc(30)
    assert (a, b, c) == (0, 30, 60) and p.alloc(20) == -1
    p.release(b, 30)
    assert p.alloc(40) == -1 and p.alloc(25) == 30
    p.release(a, 30)
    p.release(30, 25)
    p.release(c, 30)
    assert p.free == [[0, 100]] and p.used == 0


def test_all_requests_complete_with_correct_results(keys):
    clock = FakeClock()
    ex = FakeExecutor(clock, keys)
    srv = Server(ex, pool_words=4096, clock=clock)
    reqs = [mk(keys, i, i % 3, i % 2, 1 + (i * 7) % 9, arrival=0.1 * i) for i in range(30)]
    drive(srv, clock, reqs)
    assert len(srv.finished) == 30 and not srv.rejected
    for r in srv.finished:
        k = keys[r.key_id]
        x = k.d if r.kind else k.e
        assert W.limbs_to_ints(r.outputs) == [pow(v, x, k.n) for v in W.limbs_to_ints(r.inputs)]
        assert r.done >= r.arrival


def test_admission_under_memory_pressure_is_fifo(keys):
    clock = FakeClock()
    ex = FakeExecutor(clock, keys, delay=2.0)
    L = keys[0].limbs
    srv = Server(ex, pool_words=10 * L, max_inflight=2, clock=clock)
    reqs = [mk(keys, i, 0, 0, c, arrival=0.0) for i, c in enumerate([6, 5, 2, 4, 1])]
    drive(srv, clock, reqs)
    # request 1 (5 messages) cannot fit beside request 0 (6): it, and everything
    # behind it, waits; later ones never overtake it
    order = [rid for b in ex.launched for rid in b]
    assert order == sorted(order)
    assert ex.launched[0] == [0]
    assert all(srv.in_pool.used == 0 for _ in [0])


def test_oversize_request_rejected(keys):
    clock = FakeClock()
    srv = Server(FakeExecutor(clock, keys), pool_words=8 * keys[0].limbs, clock=clock)
    big = mk(keys, 0, 0, 0, 9, arrival=0.0)
    ok = mk(keys, 1, 1, 1, 3, arrival=0.0)
    drive(srv, clock, [big, ok])
    assert [r.rid for r in srv.rejected] == [0] and srv.rejected[0].error
    assert [r.rid for r in srv.finished] == [1]


def test_executor_error_fails_only_its_batch(keys):
    clock = FakeClock()
    ex = FakeExecutor(clock, keys, delay=1.0, fail_batches={1})
    srv = Server(ex, pool_words=4096, max_inflight=1, clock=clock)
    reqs = [mk(keys, i, 0, 0, 2, arrival=1.5 * i) for i in range(4)]
    drive(srv, clock, reqs)
    failed = {r.rid for r in srv.finished if r.error}
    assert failed == set(ex.launched[1]) and len(failed) >= 1
    assert all(r.outputs is not None for r in srv.finished if r.rid not in failed)
    assert srv.in_pool.used == 0 and srv.out_pool.used == 0


def test_poisson_generator_shapes(keys):
    reqs = poisson_requests(100.0, 200, 5, [k.limbs for k in keys], [k.n for k in keys], max_msgs=16)
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) >= 0) and 1.0 < arr[-1] < 3.0
    assert all(1 <= len(r.inputs) <= 16 for r in reqs)
    frac = np.mean([r.kind for r in reqs])
    assert 0.55 < frac < 0.85
