"""The continuous-batching server on the GPU: every request's result equals
the oracle's, and equals the same request run alone (tolerance 0)."""
import numpy as np
import pytest

from paper_1407_1465_amd import workloads as W
from gpu_util import oracle_modexp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_1465_amd import rsagpu  # noqa: E402
from paper_1407_1465_amd.serve import GpuExecutor, Request, Server, poisson_requests  # noqa: E402


@pytest.fixture(scope="module")
def keyset():
    keys = W.make_keys(512, 600, 3) + W.make_keys(1024, 601, 2)
    ks = rsagpu.KeySet(len(keys))
    for k in keys:
        ks.add(k.limbs, k.n, k.e, k.p, k.q, k.dp, k.dq, k.qinv)
    yield keys, ks
    ks.close()


def serve(keys, ks, reqs, pool_words=1 << 16, max_ops=4096):
    ex = GpuExecutor(ks, [k.limbs for k in keys], pool_words, max_ops)
    srv = Server(ex, pool_words, max_inflight=2, max_ops=max_ops)
    srv.run(reqs)
    return srv


def expected(keys, r):
    k = keys[r.key_id]
    x = k.d if r.kind else k.e
    return oracle_modexp(r.inputs, W.int_to_limbs(x, k.limbs), W.int_to_limbs(k.n, k.limbs))


def test_served_results_match_oracle_and_alone(keyset):
    keys, ks = keyset
    reqs = poisson_requests(2000.0, 48, 11, [k.limbs for k in keys], [k.n for k in keys], max_msgs=24)
    srv = serve(keys, ks, reqs)
    assert len(srv.finished) == len(reqs) and not srv.rejected
    assert all(r.error is None for r in srv.finished)
    by_id = {r.rid: r for r in srv.finished}
    for r in reqs[:12]:
        assert np.array_equal(by_id[r.rid].outputs, expected(keys, r)), "request %d" % r.rid
    # the same requests alone, one server each
    for r in reqs[:6]:
        alone = Request(0, r.key_id, r.kind, r.inputs, arrival=0.0)
        srv1 = serve(keys, ks, [alone])
        assert np.array_equal(srv1.finished[0].outputs, by_id[r.rid].outputs)
    assert rsagpu.device_errors() == 0
    st = srv.stats()
    assert st["requests"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0


def test_memory_pressure_on_gpu(keyset):
    keys, ks = keyset
    reqs = poisson_requests(0.0, 20, 12, [k.limbs for k in keys], [k.n for k in keys], max_msgs=16)
    srv = serve(keys, ks, reqs, pool_words=40 * 32)       # room for a few requests at a time
    assert len(srv.finished) + len(srv.rejected) == len(reqs)
    for r in srv.finished:
        assert r.error is None
        assert np.array_equal(r.outputs, expected(keys, r))
    assert srv.in_pool.used == 0


def test_serving_config_keys_match_oracle_and_alone():
    """Keys of the serving workload (2048- and 4096-bit, cached seeds), 70%
    CRT decryptions, requests of 1..64 messages arriving while batches run on
    several streams: every request against the oracle, a few alone."""
    keys = W.make_keys(2048, W.SEED_BASE + 5, 256)[:6] + W.make_keys(4096, W.SEED_BASE + 5, 64)[:3]
    ks = rsagpu.KeySet(len(keys))
    for k in keys:
        ks.add(k.limbs, k.n, k.e, k.p, k.q, k.dp, k.dq, k.qinv)
    limbs = [k.limbs for k in keys]
    reqs = poisson_requests(3000.0, 40, 21, limbs, [k.n for k in keys], max_msgs=64)
    pool, max_ops = 1 << 20, 1 << 14
    ex = GpuExecutor(ks, limbs, pool, max_ops, streams=3)
    srv = Server(ex, pool, max_inflight=ex.max_inflight, max_ops=max_ops)
    srv.run(reqs)
    assert len(srv.finished) == len(reqs) and all(r.error is None for r in srv.finished)
    for r in srv.finished:
        assert np.array_equal(r.outputs, expected(keys, r)), "request %d" % r.rid
    by_id = {r.rid: r for r in srv.finished}
    for r in reqs[:4]:
        alone = Server(ex, pool, max_inflight=1, max_ops=max_ops)
        alone.run([Request(0, r.key_id, r.kind, r.inputs, arrival=0.0)])
        assert np.array_equal(alone.finished[0].outputs, by_id[r.rid].outputs)
    assert rsagpu.device_errors() == 0
    ks.close()
