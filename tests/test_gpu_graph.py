"""The entry points captured in a HIP graph (torch.cuda.graph) and replayed:
plain CRT decryption (with its key ordering in the stream's library buffer,
or in the given order on a stream captured before it ever ran the call), plain
exponentiation and a keyset batch (with its bucket sort and the caller
stream's forked bucket streams).  Each of several replays, with eager work and synchronisation
between them, must equal the eager results."""
import numpy as np
import pytest

from paper_1407_1465_amd import workloads as W
from gpu_util import dev, crt_operands, full_operands

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_1465_amd import rsagpu  # noqa: E402


def test_graph_capture_and_replay():
    rsagpu.init()
    keys = W.make_keys(2048, 777, 4)
    L = keys[0].limbs
    count = 100                                   # several workgroups: the key ordering runs
    key_of = np.arange(count) % 4
    C = np.stack([W.uniform_below(keys[k].n, 1, 1000 + i, L)[0] for i, k in enumerate(key_of)])
    p, q, dp, dq, qi = (dev(a) for a in crt_operands(keys, key_of, L))
    c = dev(C)
    e, n = dev(full_operands(keys, key_of, L, "e")), dev(full_operands(keys, key_of, L, "n"))
    ks = rsagpu.KeySet(8)
    for k in keys:
        ks.add(k.limbs, k.n, k.e, k.p, k.q, k.dp, k.dq, k.qinv)
    offs = np.arange(count, dtype=np.int64) * L
    ops = rsagpu.pack_ops(np.ones(count, dtype=np.int64), key_of.astype(np.int64), offs, offs).cuda()
    pool_in = c.reshape(-1).clone()
    ws = torch.empty(rsagpu.ops_workspace_size(count), dtype=torch.uint8, device="cuda")

    # eager references (first use also creates the keyset's streams)
    ref_crt = rsagpu.decrypt_crt(c, p, q, dp, dq, qi)
    ref_ops = torch.zeros_like(pool_in)
    rsagpu.ops_batch(ks, ops, pool_in, ref_ops, ws)
    torch.cuda.synchronize()
    assert torch.equal(rsagpu.modexp(ref_crt, e, n), c)
    assert torch.equal(ref_ops.reshape(count, L), ref_crt)

    out_crt, out_enc, out_ops = torch.zeros_like(c), torch.zeros_like(c), torch.zeros_like(pool_in)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        # warm-up on the capture stream: the CRT call's key-order buffer for
        # this stream exists before capture (a capture never allocates)
        rsagpu.decrypt_crt(c, p, q, dp, dq, qi, out=out_crt)
        # and the keyset's fork set of this caller stream
        rsagpu.ops_batch(ks, ops, pool_in, out_ops, ws)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            rsagpu.decrypt_crt(c, p, q, dp, dq, qi, out=out_crt)
            rsagpu.modexp(out_crt, e, n, out=out_enc)
            rsagpu.ops_batch(ks, ops, pool_in, out_ops, ws)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        for t in (out_crt, out_enc, out_ops):
            t.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_crt, ref_crt)
        assert torch.equal(out_enc, c)
        assert torch.equal(out_ops, ref_ops)
        eager = rsagpu.decrypt_crt(c, p, q, dp, dq, qi)
        torch.cuda.synchronize()
        assert torch.equal(eager, ref_crt)
    assert rsagpu.device_errors() == 0
    del g

    # a stream that never ran the CRT call: the captured call allocates
    # nothing and keeps the given order; the results are the same
    g2 = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    out2 = torch.zeros_like(c)
    with torch.cuda.stream(s2):
        with torch.cuda.graph(g2, stream=s2):
            rsagpu.decrypt_crt(c, p, q, dp, dq, qi, out=out2)
    torch.cuda.current_stream().wait_stream(s2)
    for _ in range(2):
        out2.zero_()
        g2.replay()
        torch.cuda.synchronize()
        assert torch.equal(out2, ref_crt)
    del g2
    assert rsagpu.device_errors() == 0
    ks.close()
