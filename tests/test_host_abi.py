"""Host-only checks of libfwigrad: it loads, exports every function the
header declares, its schedule equals the oracle's, its codec bound equals the
oracle's, and argument errors come back as status codes (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import codec as ocodec
from oracle import revolve

F = pytest.importorskip("paper_2009_12623_amd.fwigrad")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fwigrad.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    L = F.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert sorted(F.EXPORTS) == names


@pytest.mark.parametrize("N,s", [(1, 0), (5, 1), (10, 2), (37, 3), (60, 6), (200, 10),
                                 (500, 10), (120, 119), (300, 1000)])
def test_schedule_equals_oracle(N, s):
    acts, nf = F.fwi_revolve_plan(N, s)
    ref = revolve.schedule(N, s)
    assert acts == ref
    assert nf == revolve.T_closed(N, min(s, N)) == revolve.forward_steps(ref)


def test_schedule_large_counts():
    for N, s in [(2000, 40), (3000, 40), (1500, 40)]:
        _, nf = F.fwi_revolve_plan(N, s)
        assert nf == revolve.T_closed(N, s)


@pytest.mark.parametrize("shape", [(1, 1), (4, 4), (181, 181), (1081, 481), (4, 4, 4),
                                   (5, 9, 13), (256, 256, 256), (961, 961, 367)])
def test_codec_bound_equals_oracle(shape):
    assert F.ckpt_bound(shape) == ocodec.bound(shape)


def test_bad_arguments_are_status_codes():
    L = F.lib()
    n = ctypes.c_int()
    assert L.fwi_revolve_plan(0, 3, None, 0, ctypes.byref(n), None) == F.FWI_EINVAL
    assert L.fwi_revolve_plan(10, -1, None, 0, ctypes.byref(n), None) == F.FWI_EINVAL
    assert L.fwi_revolve_plan(10, 2, None, 0, ctypes.byref(n), None) == F.FWI_ECAPACITY
    out = ctypes.c_size_t()
    dims = (ctypes.c_int * 3)(4, 0, 4)
    assert L.ckpt_bound(3, dims, ctypes.byref(out)) == F.FWI_EINVAL
    assert L.ckpt_bound(4, dims, ctypes.byref(out)) == F.FWI_EINVAL
    assert b"dims" in L.fwi_last_error() or len(L.fwi_last_error()) > 0
    # batched codec calls: a null context or null arrays are refused before any device call
    nb = (ctypes.c_size_t * 1)()
    assert L.ckpt_compress_batch(None, 1, 3, dims, None, 1e-4, None, None, nb, None) == F.FWI_EINVAL
    assert L.ckpt_decompress_batch(None, 1, 3, dims, None, nb, None, None) == F.FWI_EINVAL
    tr = F.fwi_tune_result()
    assert L.fwi_autotune_batch(None, 1, None, None, None, 2, ctypes.byref(tr), None) == F.FWI_EINVAL


def test_context_creation_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    rc = F.lib().fwi_ctx_create(ctypes.byref(h), 0, 0)
    assert rc in (F.FWI_EHIP, F.FWI_EINVAL)


def test_ckpt_pool_bytes():
    """exact need = 2 levels x slots in use x one padded level; the
    compressed worst case covers 2 x slots streams of ckpt_bound bytes; both
    grow with the slots the schedule uses and stop at nt slots"""
    import synth
    shot = synth.tiny_shot(2, n=50, so=8, nbl=6, nt=40)
    comp = shot.comp_shape
    e = [F.ckpt_pool_bytes(shot, s, False) for s in (0, 1, 3, 7, 40, 80)]
    assert e[0] == 0 and e[1] > 0
    assert e == sorted(e) and e[-1] == e[-2]
    assert e[1] % 2 == 0 and e[1] // 2 >= 4 * comp[0] * comp[1]   # one padded level
    for s in (1, 3, 7):
        used = max((a for op, a, *_ in F.fwi_revolve_plan(40, s)[0] if op == "takeshot"),
                   default=-1) + 1
        assert e[[0, 1, 3, 7].index(s)] == used * e[1]
        w = F.ckpt_pool_bytes(shot, s, True)
        assert w >= 2 * used * F.ckpt_bound(comp)
    bad = synth.Shot(2, (0, 10), 10.0, 8, 6, 40, 1e-3, 2500.0, 10.0, (0, 0), shot.rec)
    with pytest.raises(F.FwiError):
        F.ckpt_pool_bytes(bad, 3, False)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """no CPU fallback: without the built library every call path raises"""
    monkeypatch.setattr(F, "_lib", None)
    monkeypatch.setattr(F, "LIB_PATH", str(tmp_path / "libfwigrad.so"))
    with pytest.raises(RuntimeError, match="not built"):
        F.lib()
    with pytest.raises(RuntimeError, match="not built"):
        F.fwi_revolve_plan(10, 2)
