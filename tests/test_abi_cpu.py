"""The C ABI on a host without a GPU: the library loads, exports every symbol
include/rsagpu.h declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "rsagpu.h")
LIB = os.path.join(ROOT, "paper_1407_1465_amd", "librsagpu.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsa_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librsagpu.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "rsa_modexp_batch" in names and "rsa_decrypt_crt_batch" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_1407_1465_amd import rsagpu
    assert sorted(rsagpu.EXPORTS) == declared_functions()


def test_host_side_validation(lib):
    P = ctypes.c_void_p
    f = lib.rsa_modexp_batch
    f.argtypes = [P, P, P, P, ctypes.c_size_t, ctypes.c_int, P]
    dummy = P(16)
    assert f(dummy, dummy, dummy, dummy, 4, 0, None) == -2          # limbs too small
    assert f(dummy, dummy, dummy, dummy, 4, 129, None) == -2        # limbs too large
    assert f(None, dummy, dummy, dummy, 4, 8, None) == -1           # null pointer
    assert f(None, None, None, None, 0, 8, None) == 0               # empty batch
    g = lib.rsa_decrypt_crt_batch
    g.argtypes = [P] * 7 + [ctypes.c_size_t, ctypes.c_int, P]
    assert g(*([dummy] * 7), 4, 63, None) == -2                     # odd width
    assert g(*([dummy] * 6), None, 4, 64, None) == -1
    assert g(*([None] * 7), 0, 64, None) == 0
    h = lib.rsa_decrypt_crt_batch_static
    h.argtypes = [P] * 7 + [ctypes.c_size_t, ctypes.c_int, P]
    assert h(*([dummy] * 7), 4, 63, None) == -2                     # odd width
    assert h(*([dummy] * 6), None, 4, 64, None) == -1
    assert h(*([None] * 7), 0, 64, None) == 0
    assert h(*([dummy] * 7), (1 << 20) + 1, 64, None) == -1         # beyond the static scratch
    s = lib.rsa_status_str
    s.restype = ctypes.c_char_p
    assert s(0) == b"ok" and s(-2) == b"limb width out of range"
    assert lib.rsa_version() >= 100


def test_plans_are_consistent():
    from paper_1407_1465_amd import rsagpu
    for limbs in range(1, 129):
        for kind in (0, 1):
            if kind == 1 and limbs > 64:
                # no CRT half is wider than 64 words: no CRT plan there
                with pytest.raises(Exception):
                    rsagpu.get_plan(limbs, kind)
                continue
            p = rsagpu.get_plan(limbs, kind)
            assert p.radix_bits * p.padded_limbs >= 32 * limbs
            assert p.lanes_per_op * p.limbs_per_lane == p.padded_limbs
            assert p.limbs_per_lane >= 2 and 64 % p.lanes_per_op == 0
            assert p.lds_bytes <= 64 * 1024
    with pytest.raises(Exception):
        rsagpu.get_plan(0, 0)
    # overrides: a compiled instance is accepted, anything else refused
    default = rsagpu.get_plan(32, 1)
    rsagpu.set_plan(32, 1, 32, 8, 2)
    p = rsagpu.get_plan(32, 1)
    assert (p.radix_bits, p.padded_limbs, p.lanes_per_op, p.window_bits) == (32, 32, 8, 2)
    rsagpu.set_plan(32, 1, 29, 2, 3)
    p = rsagpu.get_plan(32, 1)
    assert (p.radix_bits, p.padded_limbs, p.lanes_per_op, p.window_bits) == (29, 36, 2, 3)
    for bad in ((32, 1, 29, 3, 3), (32, 1, 31, 4, 3), (32, 1, 32, 4, 1), (32, 1, 32, 2, 6), (8, 0, 29, 2, 3)):
        with pytest.raises(Exception):
            rsagpu.set_plan(*bad)
    rsagpu.set_plan(32, 1, 0, 0, 0)
    assert rsagpu.get_plan(32, 1) == default


def test_ops_batch_plans_are_separate():
    """Kinds 2, 3 and 4 (operations inside rsa_ops_batch) have their own
    plans: overriding one leaves the plain-call plan (kinds 0 and 1) alone."""
    from paper_1407_1465_amd import rsagpu
    plain = rsagpu.get_plan(32, 1)
    try:
        rsagpu.set_plan(32, 3, 29, 4, 3)
        assert rsagpu.get_plan(32, 1) == plain
        p = rsagpu.get_plan(32, 3)
        assert (p.radix_bits, p.lanes_per_op, p.window_bits) == (29, 4, 3)
        rsagpu.set_plan(64, 2, 29, 8, 2)
        assert rsagpu.get_plan(64, 2).lanes_per_op == 8
    finally:
        rsagpu.set_plan(32, 3, 0, 0, 0)
        rsagpu.set_plan(64, 2, 0, 0, 0)
    # kind 4: the widest CRT bucket of a bulk ops batch; 4096-bit halves on
    # 8 lanes there (every CRT bucket of a bulk batch runs two wave pairs per
    # workgroup), on 16 lanes (S = 80) in other ops batches and in the plain
    # CRT call (there with a 5-bit window)
    p4, p3, p1 = rsagpu.get_plan(64, 4), rsagpu.get_plan(64, 3), rsagpu.get_plan(64, 1)
    assert (p4.radix_bits, p4.padded_limbs, p4.lanes_per_op, p4.window_bits) == (29, 72, 8, 4)
    assert (p3.radix_bits, p3.padded_limbs, p3.lanes_per_op) == (29, 80, 16)
    assert (p1.lanes_per_op, p1.window_bits) == (16, 5)
    rsagpu.set_plan(64, 4, 29, 16, 4)
    try:
        assert rsagpu.get_plan(64, 3) == p3                    # kinds 3 and 4 are set apart
    finally:
        rsagpu.set_plan(64, 4, 0, 0, 0)
    assert rsagpu.get_plan(64, 4) == p4
    for kind in (-1, 5):
        with pytest.raises(Exception):
            rsagpu.get_plan(32, kind)
        with pytest.raises(Exception):
            rsagpu.set_plan(32, kind, 29, 4, 3)


def test_crt_plans_fit_the_workgroup_lds():
    """The plain CRT call (kind 1) and the bucket ending a bulk ops batch
    (kind 4) run two pairs of waves per workgroup where a half has 8 or 16
    lanes: their window tables must fit 160 KiB four times over (plus 16
    bytes).  The other ops-batch CRT buckets (kind 3) run one pair (twice
    over), and plain exponentiation one wave."""
    from paper_1407_1465_amd import rsagpu
    try:
        for kind in (1, 4):
            rsagpu.set_plan(64, kind, 29, 16, 5)                    # 2048-bit halves: 4 x 20480 bytes
            with pytest.raises(Exception):
                rsagpu.set_plan(64, kind, 29, 16, 6)                # 4 x 40960 + 16 > 160 KiB
        rsagpu.set_plan(64, 3, 29, 16, 6)                           # 2 x 40960 + 16
        rsagpu.set_plan(48, 1, 29, 8, 5)                            # 1536-bit halves: 4 x 28672
        with pytest.raises(Exception):
            rsagpu.set_plan(48, 1, 29, 8, 6)                        # 4 x 57344
        rsagpu.set_plan(32, 1, 29, 2, 4)                            # one pair: 2 x 36864
        rsagpu.set_plan(64, 0, 29, 16, 6)                           # one wave: 40960
        assert rsagpu.get_plan(64, 0).lds_bytes == 40960
        for limbs, kind in ((64, 1), (64, 3), (64, 4), (48, 1), (32, 1), (64, 0)):
            rsagpu.set_plan(limbs, kind, 0, 0, 0)
        # every default CRT plan fits
        for width in range(1, 65):
            for kind in (1, 3, 4):
                p = rsagpu.get_plan(width, kind)
                pairs = 2 if kind in (1, 4) and p.lanes_per_op >= 8 else 1
                assert 2 * pairs * p.lds_bytes + 16 <= 160 * 1024, (width, kind, p)
    finally:
        for limbs, kind in ((64, 1), (64, 3), (64, 4), (48, 1), (32, 1), (64, 0)):
            rsagpu.set_plan(limbs, kind, 0, 0, 0)


def test_plain_exponentiation_defaults_leave_room_for_two_waves_per_simd():
    """A plain exponentiation workgroup is one wave; every default plan's
    LDS lets a CU hold eight (two per SIMD), so a batch past one wave per
    SIMD does not wait for a second round."""
    from paper_1407_1465_amd import rsagpu
    for width in range(1, 129):
        p = rsagpu.get_plan(width, 0)
        assert 8 * p.lds_bytes <= 160 * 1024, (width, p)


def test_plan_lds_sizes():
    """LDS per 64-lane workgroup for a sliding window of w bits: the 2^(w-1)
    odd powers, plus one operand buffer where the multiplier is read from LDS
    (all but the radix-2^29 plans with 2 or 4 lanes), at least 4 buffers of
    S*(64/G) words."""
    from paper_1407_1465_amd import rsagpu
    cases = [
        ((32, 1, 29, 2, 4), 8 * 36 * 32 * 4),     # register multipliers, 8 odd powers
        ((32, 1, 29, 2, 3), 4 * 36 * 32 * 4),     # minimum of 4 buffers
        ((32, 1, 29, 4, 5), 16 * 36 * 16 * 4),    # 16 odd powers
        ((32, 1, 32, 8, 4), 9 * 32 * 8 * 4),      # LDS multipliers: 8 odd powers + operand buffer
        ((64, 0, 29, 8, 3), 5 * 72 * 8 * 4),      # 4 odd powers + operand buffer
        ((64, 0, 29, 8, 2), 4 * 72 * 8 * 4),      # minimum of 4 buffers
    ]
    try:
        for args, lds in cases:
            rsagpu.set_plan(*args)
            assert rsagpu.get_plan(args[0], args[1]).lds_bytes == lds, args
    finally:
        for limbs, kind in ((32, 1), (64, 0)):
            rsagpu.set_plan(limbs, kind, 0, 0, 0)


PEAK_HEADER = os.path.join(ROOT, "include", "mulpeak.h")
PEAK_LIB = os.path.join(ROOT, "paper_1407_1465_amd", "libmulpeak.so")


def test_mulpeak_library_exports_and_validates():
    """The multiply-rate probe library loads, exports what include/mulpeak.h
    declares and rejects bad arguments before any HIP call."""
    if not os.path.exists(PEAK_LIB):
        pytest.fail("libmulpeak.so is not built (run __graft_entry__.build())")
    text = re.sub(r"/\*.*?\*/", "", open(PEAK_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(mulpeak_[a-z0-9_]+)\s*\(", text)))
    assert names == ["mulpeak_launch"]
    plib = ctypes.CDLL(PEAK_LIB)
    f = plib.mulpeak_launch
    P = ctypes.c_void_p
    f.argtypes = [ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int, P]
    d = P(16)
    assert f(3, d, d, 1, 1, None) == -1          # unknown operation
    assert f(0, None, d, 1, 1, None) == -1       # null seed
    assert f(0, d, d, 0, 1, None) == -1          # no blocks
    assert f(1, d, d, 1, 0, None) == -1          # no iterations
    from paper_1407_1465_amd import mulpeak
    assert mulpeak.LANES == 256 and mulpeak.CHAINS == 16 and mulpeak.SEED_WORDS == 256
    for name, val in (("MULPEAK_LANES", 256), ("MULPEAK_CHAINS", 16), ("MULPEAK_SEED_WORDS", 256)):
        assert re.search(r"#define %s %d\b" % (name, val), text)


def test_candidate_plans_are_compiled_instances():
    """The batch tuner's candidates for a class are exactly the plans the
    library accepts (host-only calls), and the current plan is restored."""
    from paper_1407_1465_amd import rsagpu, tune
    before = rsagpu.get_plan(32, 3)
    cands = tune.candidate_plans(32, 3)
    assert rsagpu.get_plan(32, 3) == before
    assert (29, 2, 4) in cands and (32, 4, 3) in cands
    assert all(r in (29, 32) and 64 % g == 0 and 2 <= w <= 6 for r, g, w in cands)
    assert not any(r == 29 and g == 8 for r, g, _ in cands)      # no radix-2^29 8-lane 36-limb instance
    # wide classes have no CRT plans at all
    assert tune.candidate_plans(96, 3) == []
    assert len(tune.candidate_plans(128, 2)) > 0
