"""CPU ORACLE (test infrastructure only) -- codec stream wrappers.

The arithmetic lives in ``codec.c`` (see its header for the stream
definition); this module only moves numpy buffers across the C boundary.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import dims, lib, ptr

EINVAL, ECAPACITY, ECORRUPT, ENONFINITE, ERANGE = -1, -3, -4, -5, -8


class CodecError(RuntimeError):
    def __init__(self, code):
        super().__init__("oracle codec error %d" % code)
        self.code = code


def bound(shape) -> int:
    return int(lib().or_codec_bound(len(shape), dims(shape)))


def compress(x: np.ndarray, atol: float) -> bytes:
    x = np.ascontiguousarray(x, dtype=np.float32)
    cap = bound(x.shape)
    out = np.zeros(cap, dtype=np.uint8)
    n = lib().or_compress(ptr(x, ctypes.c_float), x.ndim, dims(x.shape),
                          float(atol), ptr(out, ctypes.c_uint8), cap)
    if n < 0:
        raise CodecError(n)
    return out[:n].tobytes()


def decompress(stream: bytes, shape) -> np.ndarray:
    buf = np.frombuffer(stream, dtype=np.uint8).copy()
    x = np.zeros(shape, dtype=np.float32)
    rc = lib().or_decompress(ptr(buf, ctypes.c_uint8), len(buf),
                             ptr(x, ctypes.c_float), len(shape), dims(shape))
    if rc != 0:
        raise CodecError(rc)
    return x


def header(stream: bytes) -> dict:
    b = np.frombuffer(stream[:64], dtype=np.uint8)
    u32 = lambda o: int.from_bytes(bytes(b[o:o + 4]), "little")
    u64 = lambda o: int.from_bytes(bytes(b[o:o + 8]), "little")
    return {
        "magic": bytes(b[:4]), "version": int(b[4]), "ndim": int(b[6]),
        "Q": int(b[7]), "dims": (u32(8), u32(12), u32(16)), "guard": int(b[20]),
        "log2k": int(b[21]), "tp": int(b[22]),
        "atol": np.frombuffer(bytes(b[24:32]), "<f8")[0],
        "minexp": int(np.frombuffer(bytes(b[32:36]), "<i4")[0]),
        "nchunks": u32(36), "nblocks": u64(40), "payload_bits": u64(48),
        "total_bytes": u64(56),
    }


def lift_fwd(v) -> np.ndarray:
    a = np.array(v, dtype=np.int32).copy()
    lib().or_lift_fwd4(ptr(a, ctypes.c_int32), 1)
    return a


def lift_inv(v) -> np.ndarray:
    a = np.array(v, dtype=np.int32).copy()
    lib().or_lift_inv4(ptr(a, ctypes.c_int32), 1)
    return a


def block_fwd(blk: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(blk, dtype=np.int32).copy()
    lib().or_block_fwd(a.ndim, ptr(a, ctypes.c_int32))
    return a


def block_inv(blk: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(blk, dtype=np.int32).copy()
    lib().or_block_inv(a.ndim, ptr(a, ctypes.c_int32))
    return a
