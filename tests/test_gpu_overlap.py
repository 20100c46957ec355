"""Codec overlap (fwi_ctx_set_overlap): compressed schedules run their
encodes and decodes on a second stream beside the stencil steps.  Results
must equal the single-stream run bit for bit, for store-all and
recomputing schedules, with graphs, on a user stream, and through the
split (tape) form, with unrelated work in between."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_2009_12623_amd.fwigrad")

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def problem(ndim, n, so, nt, seed=3):
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=5, nt=nt)
    v0, vt = synth.tiny_models(shot.shape, seed=seed)
    m0 = dev(synth.slowness2(synth.extend(v0, shot.nbl)).astype(np.float32))
    mt = dev(synth.slowness2(synth.extend(vt, shot.nbl)).astype(np.float32))
    return shot, m0, mt, dev(shot.wavelet().astype(np.float32))


@pytest.mark.parametrize("ndim,n,so,nt,nslots", [(3, 30, 8, 60, 60), (3, 26, 4, 70, 7), (2, 90, 16, 80, 80),
                                                 (2, 70, 8, 90, 5), (3, 40, 8, 50, 50)])
def test_overlap_equals_single_stream(ndim, n, so, nt, nslots):
    c = F.Context(0, pool_bytes=1 << 29)
    shot, m0, mt, q = problem(ndim, n, so, nt)
    d = c.forward(shot, mt, q)
    c.set_overlap(False)
    phi0, g0 = c.gradient(shot, m0, q, d, nslots=nslots, compress=True, atol=1e-4)
    c.set_overlap(True)
    for _ in range(3):
        phi, g = c.gradient(shot, m0, q, d, nslots=nslots, compress=True, atol=1e-4)
        assert torch.equal(g, g0) and phi == phi0
        x = (m0 * 3).sum()         # unrelated eager work
        assert torch.isfinite(x)
    c.close()


def test_overlap_with_graphs_and_user_stream():
    c = F.Context(0, pool_bytes=1 << 29)
    shot, m0, mt, q = problem(3, 28, 8, 60)
    d = c.forward(shot, mt, q)
    c.set_overlap(False)
    phi0, g0 = c.gradient(shot, m0, q, d, nslots=60, compress=True, atol=1e-4)
    c.set_overlap(True)
    c.set_graphs(True)
    g = torch.empty_like(m0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    for i in range(3):
        g.fill_(float("nan"))
        with torch.cuda.stream(s):
            phi, _ = c.gradient(shot, m0, q, d, nslots=60, compress=True, atol=1e-4, grad=g)
        s.synchronize()
        assert torch.equal(g, g0) and phi == phi0, i
        c.forward(shot, m0, q)
        torch.cuda.synchronize()
    for i in range(2):
        g.fill_(float("nan"))
        phi, _ = c.gradient(shot, m0, q, d, nslots=60, compress=True, atol=1e-4, grad=g)
        torch.cuda.synchronize()
        assert torch.equal(g, g0), i
    c.close()


def test_overlap_tape_form():
    c = F.Context(0, pool_bytes=1 << 29)
    shot, m0, mt, q = problem(3, 26, 8, 50)
    d_obs = c.forward(shot, mt, q)
    c.set_overlap(False)
    d0, tape0 = c.forward_ckpt(shot, m0, q, nslots=50, compress=True, atol=1e-4)
    g0 = c.backward(tape0, d0 - d_obs)
    c.set_overlap(True)
    d1, tape1 = c.forward_ckpt(shot, m0, q, nslots=50, compress=True, atol=1e-4)
    torch.cuda.synchronize()
    g1 = c.backward(tape1, d1 - d_obs)
    assert torch.equal(d1, d0) and torch.equal(g1, g0)
    c.close()


@pytest.mark.parametrize("nslots", [40, 6])
def test_overlap_batched_equals_single_stream(nslots):
    c = F.Context(0, pool_bytes=1 << 29)
    probs = [problem(3, n, 8, nt=40, seed=s) for n, s in ((16, 1), (23, 2), (19, 3))]
    shots = [p[0] for p in probs]
    m0s = [p[1] for p in probs]
    q = probs[0][3]
    dobs = [c.forward(s, mt, q) for s, _, mt, _ in probs]
    c.set_overlap(False)
    phis0, g0 = c.gradient_batch(shots, m0s, q, dobs, nslots=nslots, compress=True, atol=1e-4)
    d0, tape0 = c.forward_ckpt_batch(shots, m0s, q, nslots=nslots, compress=True, atol=1e-4)
    gt0 = c.backward_batch(tape0, [a - b for a, b in zip(d0, dobs)])
    c.set_overlap(True)
    for graphs in (False, True, True):
        c.set_graphs(graphs)
        phis, g = c.gradient_batch(shots, m0s, q, dobs, nslots=nslots, compress=True, atol=1e-4)
        assert phis == phis0
        for a, b in zip(g, g0):
            assert torch.equal(a, b)
    c.set_graphs(False)
    d1, tape1 = c.forward_ckpt_batch(shots, m0s, q, nslots=nslots, compress=True, atol=1e-4)
    gt1 = c.backward_batch(tape1, [a - b for a, b in zip(d1, dobs)])
    for a, b in zip(d1, d0):
        assert torch.equal(a, b)
    for a, b in zip(gt1, gt0):
        assert torch.equal(a, b)
    c.close()
