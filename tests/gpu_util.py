"""Helpers shared by the GPU tests: device transfer and oracle batches."""
import os

import numpy as np

import oracle
from paper_1407_1465_amd import workloads as W


def dev(arr: np.ndarray):
    import torch
    a = np.ascontiguousarray(arr, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).to("cuda")


def host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def oracle_modexp(base: np.ndarray, exp: np.ndarray, mod: np.ndarray) -> np.ndarray:
    out, _, _ = oracle.modexp_batch(base, exp, mod, nthreads=min(16, os.cpu_count() or 1))
    return out


def crt_operands(keys, key_of, limbs):
    """Per-element p, q, dp, dq, qinv arrays (half width) for CRT decryption."""
    h = limbs // 2
    def col(attr):
        table = W.ints_to_limbs([getattr(k, attr) for k in keys], h)
        return np.ascontiguousarray(table[key_of])
    return col("p"), col("q"), col("dp"), col("dq"), col("qinv")


def full_operands(keys, key_of, limbs, attr):
    table = W.ints_to_limbs([getattr(k, attr) for k in keys], limbs)
    return np.ascontiguousarray(table[key_of])
