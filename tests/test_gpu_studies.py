"""The Sec. 4 experiment drivers (paper_2009_12623_amd.studies) on small
problems: shapes of their results and the orderings the mathematics fixes
(no error at factor 1 or at exact restarts, errors shrink with atol)."""
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_2009_12623_amd.fwigrad")
from paper_2009_12623_amd import studies  # noqa: E402

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def ctx():
    c = F.Context(0, pool_bytes=1 << 29)
    yield c
    c.close()


def problem(ndim, n, so, nt, seed=3):
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=5, nt=nt)
    v0, vt = synth.tiny_models(shot.shape, seed=seed)
    m0 = dev(synth.slowness2(synth.extend(v0, shot.nbl)).astype(np.float32))
    mt = dev(synth.slowness2(synth.extend(vt, shot.nbl)).astype(np.float32))
    return shot, m0, mt, dev(shot.wavelet().astype(np.float32))


def test_compressibility_and_restart(ctx):
    shot, _, mt, q = problem(3, 24, 8, nt=60)
    rows = studies.compressibility_over_time(ctx, shot, mt, q, 1e-4, every=7)
    assert [r["step"] for r in rows] == [7, 14, 21, 28, 35, 42, 49, 56, 60]
    assert all(r["cf"] > 1 for r in rows)
    rr = studies.lossy_restart(ctx, shot, mt, q, 30, [1e-2, 1e-4, 1e-5])
    assert [r["atol"] for r in rr] == [1e-2, 1e-4, 1e-5]
    assert rr[0]["final_rel_l2"] > rr[1]["final_rel_l2"] > rr[2]["final_rel_l2"]
    assert rr[0]["cf"] > rr[2]["cf"]
    assert all(r["restart_linf"] <= r["atol"] for r in rr)


def test_gradient_studies(ctx):
    shot, m0, mt, q = problem(2, 40, 8, nt=80)
    d = ctx.forward(shot, mt, q)
    ra = studies.gradient_error_vs_atol(ctx, shot, m0, q, d, [1e-1, 1e-3, 1e-5])
    assert ra[0]["rel_l2"] > ra[-1]["rel_l2"] and ra[0]["cf"] > ra[-1]["cf"]
    rs = studies.gradient_error_vs_slots(ctx, shot, m0, q, d, [3, 10, 80], [1e-2, 1e-4])
    assert len(rs) == 6
    assert rs[0]["forward_steps"] > rs[2]["forward_steps"] == shot.nt
    rf = studies.subsampling_error(ctx, shot, m0, q, d, [1, 2, 5])
    assert rf[0]["psnr_db"] == math.inf and rf[0]["rel_l2"] == 0.0
    assert rf[1]["rel_l2"] > 0 and rf[2]["cf"] == 5.0


def test_stacking(ctx):
    shot, m0, mt, q = problem(2, 40, 8, nt=50)
    shots = []
    for x in (8, 20, 31):
        s = synth.Shot(shot.ndim, shot.shape, shot.h, shot.so, shot.nbl, shot.nt, shot.dt, shot.vmax,
                       shot.f0, (x, 2), shot.rec)
        shots.append(s)
    d = [ctx.forward(s, mt, q) for s in shots]
    rows = studies.stacking_error(ctx, shots, [m0] * 3, q, d, 1e-3, 5)
    assert [r["shots"] for r in rows] == [1, 2, 3]
    assert all(0 < r["rel_l2"] < 1e-1 for r in rows)


def test_gradient_error_shape_in_atol(ctx):
    """Sec. 4 "Gradient computation": the lossy gradient's error falls as
    atol falls, and the compression factor falls with it; a tolerance below
    what float32 blocks of this wavefield can hold (values at or above
    atol 2^23 near the source) is refused, not silently missed"""
    shot, m0, mt, q = problem(2, 48, 8, nt=120)
    d = ctx.forward(shot, mt, q)
    atols = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-9]
    rows = studies.gradient_error_vs_atol(ctx, shot, m0, q, d, atols)
    assert rows[-1] == {"atol": 1e-9, "refused": "FWI_ERANGE", "nslots": shot.nt}
    rows = rows[:-1]
    err = [r["rel_l2"] for r in rows]
    cf = [r["cf"] for r in rows]
    print("atol", atols, "rel_l2", err, "cf", cf)
    assert all(b <= a * 1.5 for a, b in zip(err, err[1:]))       # no growth as atol falls
    assert err[0] > 100 * err[-1]
    assert all(b <= a for a, b in zip(cf, cf[1:]))
