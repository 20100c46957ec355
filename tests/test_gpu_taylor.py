"""Gradient linearisation (Taylor) test on the GPU path, reference vs lossy
gradient (Sec. 4 "Gradient computation", linearisation figure): for a model
perturbation dm, the remainder |Phi(m + h dm) - Phi(m) - h <g, dm>| falls
about four-fold per halving of h with the exact gradient, and the gradient
from checkpoints compressed at atol 1e-1 gives nearly the same remainders."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_2009_12623_amd.fwigrad")

DEV = "cuda:0"


def phi(c, shot, m, q, d_obs):
    r = (c.forward(shot, m, q) - d_obs).double()
    return 0.5 * float((r * r).sum())


def test_taylor_exact_and_lossy():
    c = F.Context(0, pool_bytes=1 << 29)
    shot = synth.tiny_shot(2, n=60, so=8, nbl=8, nt=200)
    v0, vt = synth.tiny_models(shot.shape, seed=5)
    tom = lambda v: torch.from_numpy(synth.slowness2(synth.extend(v, shot.nbl)).astype(np.float32)).to(DEV)
    m0, mt = tom(v0), tom(vt)
    q = torch.from_numpy(shot.wavelet().astype(np.float32)).to(DEV)
    d_obs = c.forward(shot, mt, q)
    dm = mt - m0
    phi0 = phi(c, shot, m0, q, d_obs)
    _, g_ex = c.gradient(shot, m0, q, d_obs, nslots=shot.nt)
    _, g_lo = c.gradient(shot, m0, q, d_obs, nslots=20, compress=True, atol=1e-1)
    lin_ex = float((g_ex.double() * dm.double()).sum())
    lin_lo = float((g_lo.double() * dm.double()).sum())
    hs = [2.0 ** -k for k in range(1, 6)]
    rex, rlo = [], []
    for h in hs:
        ph = phi(c, shot, m0 + h * dm, q, d_obs)
        rex.append(abs(ph - phi0 - h * lin_ex))
        rlo.append(abs(ph - phi0 - h * lin_lo))
    ratios = [a / b for a, b in zip(rex[:-1], rex[1:])]
    print("H", hs, "exact", rex, "lossy", rlo, "ratios", ratios)
    assert all(3.0 < r < 5.0 for r in ratios[:3])
    assert all(abs(a - b) <= 0.05 * a for a, b in zip(rex[:3], rlo[:3]))
    c.close()
