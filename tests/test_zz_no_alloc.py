"""The non-allocating CRT entry point (rsa_decrypt_crt_batch_static), called
through the C ABI: bit-exact equal to rsa_decrypt_crt_batch on two calls in a
row, the second with a smaller batch (the static scratch keeps the first
call's contents), on 2048-, 1024- and 4096-bit keys (the last with two p/q
wave pairs per workgroup) with ragged batch sizes, at the largest batch it
takes, and captured into a HIP graph on a stream that never ran the call,
replayed with eager work between replays."""
import numpy as np
import pytest

from paper_1407_1465_amd import workloads as W
from gpu_util import crt_operands, dev, host, oracle_modexp, full_operands

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_1465_amd import rsagpu  # noqa: E402


def crt_batch(bits, nkeys, count, seed):
    keys = W.make_keys(bits, seed, nkeys)
    L = keys[0].limbs
    key_of = (np.arange(count) * 7 + 3) % nkeys          # keys interleaved: the ordering has work to do
    C = np.stack([W.uniform_below(keys[k].n, 1, W.derive_seed(seed, i, 9), L)[0] for i, k in enumerate(key_of)])
    return keys, key_of, C, L


@pytest.mark.parametrize("bits,nkeys,first,second,seed", [(2048, 5, 1093, 301, 6148), (1024, 3, 517, 40, 5124),
                                                           (4096, 16, 203, 37, W.SEED_BASE + 4)])
def test_static_entry_point_equals_allocating_one(bits, nkeys, first, second, seed):
    rsagpu.init()
    keys, key_of, C, L = crt_batch(bits, nkeys, first, seed)
    ops = [dev(a) for a in crt_operands(keys, key_of, L)]
    c = dev(C)
    want = rsagpu.decrypt_crt(c, *ops)
    got = torch.zeros_like(c)
    rsagpu.decrypt_crt_static(c, *ops, out=got)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    # a sample against the oracle (plain c^d mod n)
    idx = np.arange(0, first, 37)
    exp = oracle_modexp(C[idx], full_operands(keys, key_of[idx], L, "d"), full_operands(keys, key_of[idx], L, "n"))
    assert np.array_equal(host(got)[idx], exp)
    # second call, smaller, different messages: nothing of the first call's
    # scratch may leak into it
    c2 = dev(np.ascontiguousarray(C[::-1][:second]))
    ops2 = [dev(np.ascontiguousarray(a[::-1][:second])) for a in crt_operands(keys, key_of, L)]
    want2 = rsagpu.decrypt_crt(c2, *ops2)
    got2 = torch.full_like(c2, -1)
    rsagpu.decrypt_crt_static(c2, *ops2, out=got2)
    torch.cuda.synchronize()
    assert torch.equal(got2, want2)
    assert rsagpu.device_errors() == 0


def test_static_entry_point_at_its_largest_batch():
    """RSA_CRT_STATIC_MAX_COUNT messages under 7 keys (64-bit moduli): the key
    order fills the whole static scratch (its padded runs would not fit, so
    it stays dense) and the result equals the allocating call's; a sample
    against the oracle."""
    rsagpu.init()
    count, nkeys = rsagpu.CRT_STATIC_MAX_COUNT, 7
    keys = W.make_keys(64, 6464, nkeys)
    L = keys[0].limbs
    key_of = (np.arange(count) * 5 + 1) % nkeys
    C = np.zeros((count, L), dtype=np.uint32)
    for j, k in enumerate(keys):
        idx = np.nonzero(key_of == j)[0]
        C[idx] = W.uniform_below(k.n, idx.size, W.derive_seed(6464, j, 9), L)
    ops = [dev(a) for a in crt_operands(keys, key_of, L)]
    c = dev(C)
    want = rsagpu.decrypt_crt(c, *ops)
    got = torch.zeros_like(c)
    rsagpu.decrypt_crt_static(c, *ops, out=got)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    idx = np.arange(0, count, 16411)
    exp = oracle_modexp(C[idx], full_operands(keys, key_of[idx], L, "d"), full_operands(keys, key_of[idx], L, "n"))
    assert np.array_equal(host(got)[idx], exp)
    assert rsagpu.device_errors() == 0


def test_static_entry_point_rejects_oversized_batch():
    c = torch.zeros((1, 64), dtype=torch.int32, device="cuda")
    h = torch.zeros((1, 32), dtype=torch.int32, device="cuda")
    lib = rsagpu.raw_lib()
    st = lib.rsa_decrypt_crt_batch_static(c.data_ptr(), h.data_ptr(), h.data_ptr(), h.data_ptr(), h.data_ptr(),
                                          h.data_ptr(), c.data_ptr(), rsagpu.CRT_STATIC_MAX_COUNT + 1, 64, None)
    assert st == -1


def test_static_entry_point_in_a_graph():
    rsagpu.init()
    keys, key_of, C, L = crt_batch(2048, 4, 333, 4200)
    ops = [dev(a) for a in crt_operands(keys, key_of, L)]
    c = dev(C)
    want = rsagpu.decrypt_crt(c, *ops)
    torch.cuda.synchronize()
    out = torch.zeros_like(c)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()                        # never ran a CRT call before the capture
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            rsagpu.decrypt_crt_static(c, *ops, out=out)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want)
        other = torch.zeros_like(c)
        rsagpu.decrypt_crt_static(c, *ops, out=other)      # eager use of the same scratch between replays
        torch.cuda.synchronize()
        assert torch.equal(other, want)
    del g
    assert rsagpu.device_errors() == 0
