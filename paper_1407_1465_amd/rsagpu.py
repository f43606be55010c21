"""Python binding of librsagpu.so (ctypes; argument marshalling only).

Every function here forwards to the C ABI declared in include/rsagpu.h.
Big integers are int32 (or uint32) torch tensors of shape (count, limbs) on a
HIP device, little-endian limbs, message-major; torch owns the memory and the
stream.  The library must have been built (``python -m
paper_1407_1465_amd.build``); a missing library raises at import.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsagpu.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("librsagpu.so is not built (run `python -m paper_1407_1465_amd.build`)")

_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_lib.rsa_modexp_batch.argtypes = [_P, _P, _P, _P, ctypes.c_size_t, ctypes.c_int, _P]
_lib.rsa_modexp_batch.restype = ctypes.c_int
_lib.rsa_decrypt_crt_batch.argtypes = [_P] * 7 + [ctypes.c_size_t, ctypes.c_int, _P]
_lib.rsa_decrypt_crt_batch.restype = ctypes.c_int
_lib.rsa_decrypt_crt_batch_static.argtypes = [_P] * 7 + [ctypes.c_size_t, ctypes.c_int, _P]
_lib.rsa_decrypt_crt_batch_static.restype = ctypes.c_int
_lib.rsa_device_errors.argtypes = [_P, ctypes.POINTER(ctypes.c_uint64)]
_lib.rsa_device_errors.restype = ctypes.c_int
_lib.rsa_status_str.argtypes = [ctypes.c_int]
_lib.rsa_status_str.restype = ctypes.c_char_p
_lib.rsa_version.argtypes = []
_lib.rsa_version.restype = ctypes.c_int


class _Plan(ctypes.Structure):
    _fields_ = [("radix_bits", ctypes.c_int), ("padded_limbs", ctypes.c_int), ("lanes_per_op", ctypes.c_int),
                ("limbs_per_lane", ctypes.c_int), ("window_bits", ctypes.c_int),
                ("lds_bytes", ctypes.c_int)]


_lib.rsa_get_plan.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Plan)]
_lib.rsa_get_plan.restype = ctypes.c_int
_lib.rsa_set_plan.argtypes = [ctypes.c_int] * 5
_lib.rsa_set_plan.restype = ctypes.c_int
_lib.rsa_autotune.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_size_t, _P, ctypes.POINTER(_Plan)]
_lib.rsa_autotune.restype = ctypes.c_int
_lib.rsa_init.argtypes = []
_lib.rsa_init.restype = ctypes.c_int

_lib.rsa_keyset_create.argtypes = [ctypes.POINTER(_P), ctypes.c_int]
_lib.rsa_keyset_create.restype = ctypes.c_int
_U32P = ctypes.POINTER(ctypes.c_uint32)
_lib.rsa_keyset_add.argtypes = [_P, ctypes.c_int] + [_U32P] * 7 + [ctypes.POINTER(ctypes.c_int32)]
_lib.rsa_keyset_add.restype = ctypes.c_int
_lib.rsa_keyset_destroy.argtypes = [_P]
_lib.rsa_keyset_destroy.restype = ctypes.c_int
_lib.rsa_ops_workspace_size.argtypes = [ctypes.c_size_t]
_lib.rsa_ops_workspace_size.restype = ctypes.c_size_t
_lib.rsa_ops_batch.argtypes = [_P, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P,
                               ctypes.c_size_t, _P]
_lib.rsa_ops_batch.restype = ctypes.c_int
_lib.rsa_keyset_set_forks.argtypes = [_P, ctypes.c_int]
_lib.rsa_keyset_set_forks.restype = ctypes.c_int

# exported symbols, in the order include/rsagpu.h declares them
EXPORTS = ("rsa_modexp_batch", "rsa_decrypt_crt_batch", "rsa_decrypt_crt_batch_static", "rsa_get_plan", "rsa_set_plan", "rsa_autotune", "rsa_init",
           "rsa_keyset_create", "rsa_keyset_add", "rsa_keyset_destroy", "rsa_ops_workspace_size",
           "rsa_ops_batch", "rsa_keyset_set_forks", "rsa_device_errors", "rsa_status_str", "rsa_version")

OP_ENCRYPT = 0
OP_DECRYPT_CRT = 1


class RSAError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s: %s (%d)" % (what, _lib.rsa_status_str(status).decode(), status))
        self.status = status


def _check(status: int, what: str) -> None:
    if status != 0:
        raise RSAError(status, what)


@dataclass
class Plan:
    radix_bits: int
    padded_limbs: int
    lanes_per_op: int
    limbs_per_lane: int
    window_bits: int
    lds_bytes: int


def get_plan(limbs: int, kind: int = 0) -> Plan:
    p = _Plan()
    _check(_lib.rsa_get_plan(limbs, kind, ctypes.byref(p)), "rsa_get_plan")
    return Plan(p.radix_bits, p.padded_limbs, p.lanes_per_op, p.limbs_per_lane, p.window_bits, p.lds_bytes)


def set_plan(limbs: int, kind: int, radix_bits: int, lanes_per_op: int, window_bits: int) -> None:
    """Override the plan of a limb width (all zero restores the default)."""
    _check(_lib.rsa_set_plan(limbs, kind, radix_bits, lanes_per_op, window_bits), "rsa_set_plan")


def autotune(limbs: int, kind: int, exp_bits: int, count: int,
             stream: Optional[torch.cuda.Stream] = None) -> Plan:
    """Times every kernel instance / window for the class and installs the fastest."""
    p = _Plan()
    _check(_lib.rsa_autotune(limbs, kind, exp_bits, count, _stream_handle(stream), ctypes.byref(p)), "rsa_autotune")
    return Plan(p.radix_bits, p.padded_limbs, p.lanes_per_op, p.limbs_per_lane, p.window_bits, p.lds_bytes)


def init() -> None:
    _check(_lib.rsa_init(), "rsa_init")


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _operand(t: torch.Tensor, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype not in (torch.int32, torch.uint32):
        raise TypeError("%s must be int32/uint32 limbs" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t


def modexp(base: torch.Tensor, exp: torch.Tensor, mod: torch.Tensor,
           out: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """out[i] = base[i] ^ exp[i] mod mod[i] (rsa_modexp_batch)."""
    _operand(base, "base")
    if base.dim() != 2:
        raise ValueError("base must be (count, limbs)")
    count, limbs = base.shape
    _operand(exp, "exp", base.shape)
    _operand(mod, "mod", base.shape)
    if out is None:
        out = torch.empty_like(base)
    _operand(out, "out", base.shape)
    _check(_lib.rsa_modexp_batch(base.data_ptr(), exp.data_ptr(), mod.data_ptr(), out.data_ptr(),
                                 count, limbs, _stream_handle(stream)), "rsa_modexp_batch")
    return out


def decrypt_crt(c: torch.Tensor, p: torch.Tensor, q: torch.Tensor, dp: torch.Tensor,
                dq: torch.Tensor, qinv: torch.Tensor, out: Optional[torch.Tensor] = None,
                stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """out[i] = c[i] ^ d mod p[i]*q[i] by CRT (rsa_decrypt_crt_batch)."""
    _operand(c, "c")
    if c.dim() != 2:
        raise ValueError("c must be (count, limbs)")
    count, limbs = c.shape
    hshape = (count, limbs // 2)
    for name, t in (("p", p), ("q", q), ("dp", dp), ("dq", dq), ("qinv", qinv)):
        _operand(t, name, hshape)
    if out is None:
        out = torch.empty_like(c)
    _operand(out, "out", c.shape)
    _check(_lib.rsa_decrypt_crt_batch(c.data_ptr(), p.data_ptr(), q.data_ptr(), dp.data_ptr(),
                                      dq.data_ptr(), qinv.data_ptr(), out.data_ptr(), count, limbs,
                                      _stream_handle(stream)), "rsa_decrypt_crt_batch")
    return out


CRT_STATIC_MAX_COUNT = 1 << 20


def decrypt_crt_static(c: torch.Tensor, p: torch.Tensor, q: torch.Tensor, dp: torch.Tensor,
                       dq: torch.Tensor, qinv: torch.Tensor, out: torch.Tensor,
                       stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """decrypt_crt into a caller-provided `out` through the entry point that
    never allocates device memory (rsa_decrypt_crt_batch_static: its scratch
    is the library's static device array, shared by every call on a device,
    so calls must not overlap in time; count <= CRT_STATIC_MAX_COUNT)."""
    _operand(c, "c")
    if c.dim() != 2:
        raise ValueError("c must be (count, limbs)")
    count, limbs = c.shape
    hshape = (count, limbs // 2)
    for name, t in (("p", p), ("q", q), ("dp", dp), ("dq", dq), ("qinv", qinv)):
        _operand(t, name, hshape)
    _operand(out, "out", c.shape)
    _check(_lib.rsa_decrypt_crt_batch_static(c.data_ptr(), p.data_ptr(), q.data_ptr(), dp.data_ptr(),
                                             dq.data_ptr(), qinv.data_ptr(), out.data_ptr(), count, limbs,
                                             _stream_handle(stream)), "rsa_decrypt_crt_batch_static")
    return out


def device_errors(stream: Optional[torch.cuda.Stream] = None) -> int:
    """Per-element data errors since the last call (synchronises the stream)."""
    v = ctypes.c_uint64(0)
    _check(_lib.rsa_device_errors(_stream_handle(stream), ctypes.byref(v)), "rsa_device_errors")
    return int(v.value)


def _host_limbs(value: int, words: int):
    arr = (ctypes.c_uint32 * words)()
    for i in range(words):
        arr[i] = (value >> (32 * i)) & 0xFFFFFFFF
    return arr


class KeySet:
    """Resident keys on the current device (rsa_keyset_*)."""

    def __init__(self, max_keys: int):
        self._h = _P()
        _check(_lib.rsa_keyset_create(ctypes.byref(self._h), max_keys), "rsa_keyset_create")
        self.limbs = []

    def add(self, limbs: int, n: int, e: int, p: int, q: int, dp: int, dq: int, qinv: int) -> int:
        """Adds a key given as Python integers; returns its key id."""
        h = limbs // 2
        kid = ctypes.c_int32(-1)
        args = [_host_limbs(n, limbs), _host_limbs(e, limbs)] + [_host_limbs(v, h) for v in (p, q, dp, dq, qinv)]
        _check(_lib.rsa_keyset_add(self._h, limbs, *[ctypes.cast(a, _U32P) for a in args], ctypes.byref(kid)),
               "rsa_keyset_add")
        self.limbs.append(limbs)
        return kid.value

    def set_forks(self, forks: int) -> None:
        """Streams a batch forks its widest CRT buckets onto (rsa_keyset_set_forks)."""
        _check(_lib.rsa_keyset_set_forks(self._h, forks), "rsa_keyset_set_forks")

    def close(self) -> None:
        if self._h:
            _check(_lib.rsa_keyset_destroy(self._h), "rsa_keyset_destroy")
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def ops_workspace_size(max_ops: int) -> int:
    return int(_lib.rsa_ops_workspace_size(max_ops))


def ops_batch(ks: KeySet, ops: torch.Tensor, in_pool: torch.Tensor, out_pool: torch.Tensor,
              workspace: torch.Tensor, nops: Optional[int] = None,
              stream: Optional[torch.cuda.Stream] = None) -> None:
    """Runs operation descriptors against a keyset (rsa_ops_batch).

    ops: int64 device tensor (nops, 3) laid out as rsa_op: column 0 holds
    kind | key_id << 32, columns 1 and 2 the input and output word offsets.
    in_pool / out_pool: int32 device tensors of 32-bit words; workspace: a
    device tensor of at least ops_workspace_size(nops) bytes."""
    if ops.dtype != torch.int64 or ops.dim() != 2 or ops.shape[1] != 3 or not ops.is_contiguous():
        raise ValueError("ops must be a contiguous (n, 3) int64 tensor")
    n = ops.shape[0] if nops is None else nops
    for name, t in (("ops", ops), ("in_pool", in_pool), ("out_pool", out_pool), ("workspace", workspace)):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("%s must be a contiguous device tensor" % name)
    _check(_lib.rsa_ops_batch(ks.handle, ops.data_ptr(), n, in_pool.data_ptr(), in_pool.numel(),
                              out_pool.data_ptr(), out_pool.numel(), workspace.data_ptr(),
                              workspace.numel() * workspace.element_size(), _stream_handle(stream)),
           "rsa_ops_batch")


def pack_ops(kinds, key_ids, in_offs, out_offs) -> torch.Tensor:
    """Host int64 (n, 3) array in the rsa_op layout."""
    import numpy as np
    kinds = np.asarray(kinds, dtype=np.int64)
    key_ids = np.asarray(key_ids, dtype=np.int64)
    a = np.empty((len(kinds), 3), dtype=np.int64)
    a[:, 0] = kinds | (key_ids << 32)
    a[:, 1] = np.asarray(in_offs, dtype=np.int64)
    a[:, 2] = np.asarray(out_offs, dtype=np.int64)
    return torch.from_numpy(a)


def version() -> int:
    return _lib.rsa_version()


def raw_lib() -> ctypes.CDLL:
    return _lib
