"""CPU ORACLE -- test infrastructure, not product code.

A plain, slow, FP64 (solver) / integer-exact (codec) reference of the
checkpointed adjoint FWI gradient with lossily compressed checkpoints.  Only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may import it.  It shares no code with the HIP path (``paper_2009_12623_amd``)
and does not import it; both take their inputs from ``synth``.

Modules: ``wave.c``/``codec.c`` (C, built here with gcc into liboracle.so),
``solver`` (time loops, adjoint, gradient, Born, checkpointed gradient),
``codec`` (stream wrappers), ``revolve`` (schedule), ``metrics``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, f) for f in ("wave.c", "codec.c")]
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle's C sources with gcc (CPU only)."""
    if not force and os.path.exists(_SO) and all(
            os.path.getmtime(_SO) >= os.path.getmtime(s) for s in _SRC):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-o", tmp] + _SRC + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        D = ctypes.POINTER(ctypes.c_double)
        F = ctypes.POINTER(ctypes.c_float)
        Lp = ctypes.POINTER(ctypes.c_long)
        I32 = ctypes.POINTER(ctypes.c_int32)
        U8 = ctypes.POINTER(ctypes.c_uint8)
        L.or_fd_coeffs.argtypes = [ctypes.c_int, D]
        L.or_laplacian.argtypes = [ctypes.c_int, Lp, ctypes.c_double, ctypes.c_int, D, D]
        L.or_damping.argtypes = [ctypes.c_int, Lp, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, D]
        L.or_step.argtypes = [ctypes.c_int, Lp, ctypes.c_double, ctypes.c_int,
                              ctypes.c_double, D, D, D, D, D, D, ctypes.c_int, Lp, D]
        L.or_image.argtypes = [ctypes.c_long, ctypes.c_double, D, D, D, D, D]
        L.or_born_rhs.argtypes = [ctypes.c_long, ctypes.c_double, D, D, D, D, D]
        L.or_codec_bound.argtypes = [ctypes.c_int, Lp]
        L.or_codec_bound.restype = ctypes.c_long
        L.or_compress.argtypes = [F, ctypes.c_int, Lp, ctypes.c_double, U8, ctypes.c_long]
        L.or_compress.restype = ctypes.c_long
        L.or_decompress.argtypes = [U8, ctypes.c_long, F, ctypes.c_int, Lp]
        L.or_lift_fwd4.argtypes = [I32, ctypes.c_int]
        L.or_lift_inv4.argtypes = [I32, ctypes.c_int]
        L.or_block_fwd.argtypes = [ctypes.c_int, I32]
        L.or_block_inv.argtypes = [ctypes.c_int, I32]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops in this thread's later calls."""
    lib()
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def dims(shape) -> ctypes.Array:
    arr = (ctypes.c_long * 3)(*(list(shape) + [1] * (3 - len(shape))))
    return arr
