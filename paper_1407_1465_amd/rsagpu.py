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
_lib.rsa_init.argtypes = []
_lib.rsa_init.restype = ctypes.c_int

# exported symbols, in the order include/rsagpu.h declares them
EXPORTS = ("rsa_modexp_batch", "rsa_decrypt_crt_batch", "rsa_get_plan", "rsa_set_plan", "rsa_init",
           "rsa_device_errors", "rsa_status_str", "rsa_version")


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


def device_errors(stream: Optional[torch.cuda.Stream] = None) -> int:
    """Per-element data errors since the last call (synchronises the stream)."""
    v = ctypes.c_uint64(0)
    _check(_lib.rsa_device_errors(_stream_handle(stream), ctypes.byref(v)), "rsa_device_errors")
    return int(v.value)


def version() -> int:
    return _lib.rsa_version()


def raw_lib() -> ctypes.CDLL:
    return _lib
