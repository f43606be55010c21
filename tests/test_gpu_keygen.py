"""Batched key generation with the Miller-Rabin rounds on the GPU: the keys
are exactly those of the CPU generator for the same seeds (same candidate
stream, same bases, first two distinct primes)."""
import pytest

from paper_1407_1465_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_1465_amd import keygen, rsagpu  # noqa: E402


@pytest.mark.parametrize("bits,count", [(64, 8), (512, 4), (2048, 2)])
def test_gpu_keygen_equals_cpu_keygen(bits, count):
    seed = 9100 + bits
    got = keygen.make_keys_gpu(bits, seed, count)
    want = [W.make_key(bits, W.derive_seed(seed, bits, j)) for j in range(count)]
    assert got == want
    assert rsagpu.device_errors() == 0


def test_gpu_miller_rabin_rounds():
    """Single rounds against known answers: primes pass every base, a
    Carmichael number and strong pseudoprimes fail where theory says."""
    limbs = 1
    p = 1000003                                   # prime
    carmichael = 561                              # 3 * 11 * 17
    spsp2 = 2047                                  # strong pseudoprime to base 2, fails base 3
    pairs = [(p, 2), (p, 3), (p, 999999), (carmichael, 2), (spsp2, 2), (spsp2, 3)]
    assert keygen.miller_rabin_gpu(pairs, limbs, rsagpu, torch) == [True, True, True, False, True, False]
