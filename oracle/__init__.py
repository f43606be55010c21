"""Plain CPU oracle for batched RSA modular exponentiation.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg import this package.  It shares no code with the
GPU library (``paper_1407_1465_amd``), and the GPU library never imports it.

The arithmetic lives in ``rsa_oracle.c`` (schoolbook multiply, Knuth
Algorithm D remainder, left-to-right binary exponentiation of the paper's
Section 3.6.3, Fig. 5).  This module only compiles it with gcc, loads it with
ctypes and converts between Python integers / numpy arrays and limb spans.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rsa_oracle.c")
_LIB = os.path.join(_HERE, "librsa_oracle.so")
_lock = threading.Lock()
_lib = None

_U32P = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/librsa_oracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
               _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
            L.oracle_bn_mul.argtypes = [_U32P, _U32P, ctypes.c_int, _U32P, ctypes.c_int]
            L.oracle_bn_mul.restype = None
            for name in ("oracle_bn_mod", "oracle_bn_mod_slow"):
                f = getattr(L, name)
                f.argtypes = [_U32P, _U32P, ctypes.c_int, _U32P, ctypes.c_int]
                f.restype = ctypes.c_int
            for name in ("oracle_modexp", "oracle_modexp_rtl"):
                f = getattr(L, name)
                f.argtypes = [_U32P, _U32P, _U32P, _U32P, ctypes.c_int]
                f.restype = ctypes.c_int
            L.oracle_modexp_naive.argtypes = [_U32P, _U32P, ctypes.c_uint64, _U32P, ctypes.c_int,
                                              _U32P]
            L.oracle_modexp_naive.restype = ctypes.c_int
            L.oracle_modexp_batch.argtypes = [_U32P, _U32P, _U32P, _U32P, ctypes.c_size_t,
                                              ctypes.c_int, ctypes.c_size_t, ctypes.c_size_t,
                                              ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
            L.oracle_modexp_batch.restype = ctypes.c_int
            _lib = L
    return _lib


# ---- conversions (the oracle's own) ---------------------------------------

def _to_span(x: int, k: int) -> np.ndarray:
    if x < 0 or x.bit_length() > 32 * k:
        raise ValueError("value does not fit in %d limbs" % k)
    return np.array([(x >> (32 * i)) & 0xFFFFFFFF for i in range(k)], dtype=np.uint32)


def _from_span(a) -> int:
    v = 0
    for i, w in enumerate(np.asarray(a, dtype=np.uint32).tolist()):
        v |= int(w) << (32 * i)
    return v


def _p(a: np.ndarray):
    return a.ctypes.data_as(_U32P)


def _limbs_for(*vals: int) -> int:
    return max(1, max((v.bit_length() + 31) // 32 for v in vals))


def _check(st: int, what: str) -> None:
    if st == -1:
        raise ZeroDivisionError("%s: zero modulus" % what)
    if st != 0:
        raise MemoryError("%s: status %d" % (what, st))


# ---- single-element API on Python integers ----------------------------------

def bn_mul(u: int, v: int) -> int:
    m, n = _limbs_for(u), _limbs_for(v)
    a, b = _to_span(u, m), _to_span(v, n)
    w = np.zeros(m + n, dtype=np.uint32)
    lib().oracle_bn_mul(_p(w), _p(a), m, _p(b), n)
    return _from_span(w)


def bn_mod(u: int, v: int, slow: bool = False) -> int:
    m, n = _limbs_for(u), _limbs_for(v)
    a, b = _to_span(u, m), _to_span(v, n)
    r = np.zeros(n, dtype=np.uint32)
    f = lib().oracle_bn_mod_slow if slow else lib().oracle_bn_mod
    _check(f(_p(r), _p(a), m, _p(b), n), "bn_mod")
    return _from_span(r)


def modexp(g: int, x: int, n: int, method: str = "ltr") -> int:
    """g^x mod n by the left-to-right ("ltr") or right-to-left ("rtl") binary method."""
    k = _limbs_for(g, x, n)
    out = np.zeros(k, dtype=np.uint32)
    bs, xs, ns = _to_span(g, k), _to_span(x, k), _to_span(n, k)
    f = lib().oracle_modexp if method == "ltr" else lib().oracle_modexp_rtl
    _check(f(_p(out), _p(bs), _p(xs), _p(ns), k), "modexp")
    return _from_span(out)


def modexp_naive(g: int, e: int, n: int, trace: bool = False):
    """g^e mod n by e-1 repeated modular products (Section 3.6.2, Fig. 4).

    With ``trace`` also returns the intermediate after each step."""
    k = _limbs_for(g, n)
    out = np.zeros(k, dtype=np.uint32)
    tr = np.zeros(max(e, 1) * k, dtype=np.uint32) if trace else None
    _check(lib().oracle_modexp_naive(_p(out), _p(_to_span(g, k)), e, _p(_to_span(n, k)), k,
                                     _p(tr) if trace else None), "modexp_naive")
    if trace:
        return _from_span(out), [_from_span(tr[i * k:(i + 1) * k]) for i in range(e)]
    return _from_span(out)


# ---- batch API on limb arrays -----------------------------------------------

def modexp_batch(base: np.ndarray, exp: np.ndarray, mod: np.ndarray, nthreads: int = 0):
    """out[i] = base[i]^exp[i] mod mod[i] on message-major uint32 arrays.

    ``base`` is (count, k); ``exp`` and ``mod`` are (count, k) or (k,) for one
    value shared by every element.  ``nthreads`` <= 0 uses every host core.
    Returns (out, wall_seconds, threads_used)."""
    base = np.ascontiguousarray(base, dtype=np.uint32)
    if base.ndim != 2:
        raise ValueError("base must be (count, limbs)")
    count, k = base.shape
    exp = np.ascontiguousarray(exp, dtype=np.uint32)
    mod = np.ascontiguousarray(mod, dtype=np.uint32)
    es = 0 if exp.ndim == 1 else k
    ms = 0 if mod.ndim == 1 else k
    if exp.shape[-1] != k or mod.shape[-1] != k:
        raise ValueError("limb widths differ")
    if es and exp.shape[0] != count or ms and mod.shape[0] != count:
        raise ValueError("element counts differ")
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    out = np.zeros((count, k), dtype=np.uint32)
    wall = ctypes.c_double(0.0)
    _check(lib().oracle_modexp_batch(_p(base), _p(exp), _p(mod), _p(out), count, k, es, ms,
                                     nthreads, ctypes.byref(wall)), "modexp_batch")
    return out, wall.value, min(nthreads, max(count, 1))
