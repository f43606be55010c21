"""ctypes binding of libmulpeak.so: the issue rate of the VALU's 32-bit
integer multiplies (v_mad_u64_u32, v_mul_lo_u32, v_mul_hi_u32), the
instructions every Montgomery product of the RSA kernels is made of.

Each launch runs blocks x 256 lanes x 16 independent chains x iters
operations (include/mulpeak.h); the rate is timed with HIP events on torch's
current stream, which is the stream the launch goes to.
"""
from __future__ import annotations

import ctypes
import os
import statistics

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmulpeak.so")
LANES, CHAINS, SEED_WORDS = 256, 16, 256
OPS = {0: "v_mad_u64_u32", 1: "v_mul_lo_u32", 2: "v_mul_hi_u32"}

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmulpeak.so is not built (run `python -m paper_1407_1465_amd.build`)")
        L = ctypes.CDLL(LIB_PATH)
        L.mulpeak_launch.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p]
        L.mulpeak_launch.restype = ctypes.c_int
        _lib = L
    return _lib


def measure(op: int, waves_per_simd: int = 8, iters: int = 8192, reps: int = 7) -> dict:
    """Median over `reps` timed launches (after one warm-up) of the rate of
    operation `op` with `waves_per_simd` waves resident on every SIMD."""
    L = lib()
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    blocks = cus * waves_per_simd          # 4 waves per workgroup, 4 SIMDs per CU
    seed = torch.randint(0, 2 ** 31 - 1, (SEED_WORDS,), dtype=torch.int32, device="cuda")
    sink = torch.empty(blocks * LANES, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def launch():
        st = L.mulpeak_launch(op, ctypes.c_void_p(seed.data_ptr()), ctypes.c_void_p(sink.data_ptr()), blocks,
                              iters, ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise RuntimeError("mulpeak_launch failed (%d)" % st)

    launch()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        launch()
        b.record(stream)
    torch.cuda.synchronize()
    ms = statistics.median(a.elapsed_time(b) for a, b in evs)
    ops = blocks * LANES * CHAINS * iters
    return {"op": OPS[op], "ops_per_s": ops / (ms / 1e3), "ms_per_launch": ms, "ops_per_launch": ops,
            "blocks": blocks, "lanes_per_block": LANES, "chains_per_lane": CHAINS, "iters": iters, "cus": cus}
