"""ckpt_compress_static: the allocation-free variant of ckpt_compress for
callers that cannot allocate (its encode workspace is a static device array
of the library).  Through the C ABI, two calls in a row (the second with a
smaller field, so the workspace holds the first call's contents) must
write the same bytes as ckpt_compress, which decode to within atol; a
field whose workspace exceeds the static array is refused."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import codec as ocodec

pytestmark = pytest.mark.gpu
F = pytest.importorskip("paper_2009_12623_amd.fwigrad")


def _static(x, atol):
    L = F.lib()
    cap = F.ckpt_bound(tuple(x.shape))
    out = torch.full((cap,), 0xA5, dtype=torch.uint8, device="cuda:0")
    nb = ctypes.c_size_t()
    rc = L.ckpt_compress_static(ctypes.c_void_p(x.data_ptr()), x.dim(), F._dims3(x.shape), float(atol),
                                ctypes.c_void_p(out.data_ptr()), cap, ctypes.byref(nb),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, out[:nb.value]


def test_static_compress_equals_ckpt_compress_twice():
    ctx = F.Context(0, pool_bytes=1 << 24)
    cases = [(synth.wavefield_like((61, 47, 83), seed=2), 1e-4),      # first: the larger field
             (synth.wavefield_like((19, 23, 12), seed=3), 1e-3),      # second: smaller, other atol
             (synth.wavefield_like((301, 257), seed=4), 1e-5)]        # 2D
    for x, atol in cases:
        xd = torch.from_numpy(x).to("cuda:0")
        rc, s = _static(xd, atol)
        assert rc == F.FWI_OK, F.lib().fwi_last_error()
        ref = ctx.compress(xd, atol)
        assert torch.equal(s, ref), (x.shape, atol)
        assert s.cpu().numpy().tobytes() == ocodec.compress(x, atol)
        y = ctx.decompress(s, x.shape).cpu().numpy()
        assert np.max(np.abs(y.astype(np.float64) - x)) <= atol
    ctx.close()


def test_static_compress_rejects_fields_beyond_its_workspace():
    big = torch.zeros((260, 260, 260), dtype=torch.float32, device="cuda:0")
    rc, _ = _static(big, 1e-4)
    assert rc == F.FWI_EINVAL
    assert b"static workspace" in F.lib().fwi_last_error()
    x = synth.wavefield_like((33, 31, 29), seed=5)
    x[3, 4, 5] = 1e9
    rc, _ = _static(torch.from_numpy(x).to("cuda:0"), 1e-4)
    assert rc == F.FWI_ERANGE
    # a valid call afterwards is unaffected by the failed ones
    x[3, 4, 5] = 0.5
    rc, s = _static(torch.from_numpy(x).to("cuda:0"), 1e-4)
    assert rc == F.FWI_OK and s.cpu().numpy().tobytes() == ocodec.compress(x, 1e-4)
