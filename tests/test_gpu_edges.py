"""Degenerate cases of the gradient path against the FP64 oracle: time axes
of 1-5 steps with 1, 2 or nt checkpoint slots (a wavelet that is large from
the first step, so every step matters), and a shot without receivers (no
data, zero objective and zero gradient), with direct launches and with
captured schedules."""
import numpy as np
import pytest
import torch

import synth
from oracle import metrics, solver

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_2009_12623_amd.fwigrad")

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def setup(ndim, nt, seed=2):
    s = synth.tiny_shot(ndim, n=20 if ndim == 2 else 12, so=4, nbl=5, nt=nt)
    v0, vt = synth.tiny_models(s.shape, seed=seed)
    m0 = synth.slowness2(synth.extend(v0, s.nbl))
    mt = synth.slowness2(synth.extend(vt, s.nbl))
    q = np.random.default_rng(seed).standard_normal(nt)
    return s, m0, mt, q


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("nt", [1, 2, 3, 5])
@pytest.mark.parametrize("compress", [False, True])
def test_short_time_axes_match_oracle(ndim, nt, compress):
    s, m0, mt, q = setup(ndim, nt)
    dobs = solver.forward(solver.Problem(s, mt, wavelet=q))
    phi_ref, gref, _ = solver.gradient(solver.Problem(s, m0, wavelet=q), dobs)
    assert phi_ref > 0 and np.abs(gref).max() > 0
    c = F.Context(0, pool_bytes=1 << 26)
    for nslots in sorted({1, 2, nt}):
        if nslots > nt:
            continue
        phi, g = c.gradient(s, dev(m0.astype(np.float32)), dev(q.astype(np.float32)),
                            dev(dobs.astype(np.float32)), nslots=nslots, compress=compress, atol=1e-4)
        assert abs(phi - phi_ref) <= 1e-4 * phi_ref, (nslots, phi, phi_ref)
        assert metrics.rel_l2(g.cpu().numpy(), gref) <= 1e-4, nslots
    c.close()


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("compress", [False, True])
def test_shot_without_receivers(graphs, compress):
    base, m0, _, q = setup(2, 30)
    s = synth.Shot(2, base.shape, base.h, base.so, base.nbl, base.nt, base.dt, base.vmax, base.f0, base.src,
                   np.zeros((0, 2), np.int32))
    c = F.Context(0, pool_bytes=1 << 26)
    c.set_graphs(graphs)
    mg, qg = dev(m0.astype(np.float32)), dev(q.astype(np.float32))
    d = c.forward(s, mg, qg)
    assert tuple(d.shape) == (30, 0)
    for _ in range(2):
        phi, g = c.gradient(s, mg, qg, d, nslots=4, compress=compress, atol=1e-4)
        assert phi == 0.0
        assert torch.count_nonzero(g).item() == 0
    ds, tape = c.forward_ckpt(s, mg, qg, nslots=4, compress=compress, atol=1e-4, pool_bytes=1 << 24)
    g2 = c.backward(tape, ds)
    tape.free()
    assert torch.count_nonzero(g2).item() == 0
    c.close()
