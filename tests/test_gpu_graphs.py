"""Captured schedules (fwi_ctx_set_graphs): the first call with a signature
captures the whole checkpoint schedule into a hipGraph, later calls replay
it.  Every replay must equal the direct-launch result bit for bit, with
unrelated eager work and synchronisations between the replays, and a graph
must be re-captured after the library reallocates a buffer it refers to.
"""
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


@pytest.mark.parametrize("ndim,n,so,compress", [(2, 50, 16, True), (2, 50, 8, False),
                                                (3, 18, 8, True), (3, 18, 4, False)])
def test_graph_replays_equal_direct(ndim, n, so, compress):
    c = F.Context(0, pool_bytes=1 << 28)
    shot, m0, mt, q = problem(ndim, n, so, nt=45)
    other, om, _, oq = problem(ndim, n + 3, so, nt=20, seed=5)
    d = c.forward(shot, mt, q)
    phi0, g0 = c.gradient(shot, m0, q, d, nslots=4, compress=compress, atol=1e-4)
    n0 = c.stats()["n_forward"]
    c.set_graphs(True)
    g = torch.empty_like(m0)
    for i in range(4):
        g.fill_(float("nan"))
        phi, _ = c.gradient(shot, m0, q, d, nslots=4, compress=compress, atol=1e-4, grad=g)
        assert torch.equal(g, g0), i
        assert phi == phi0
        assert c.stats()["n_forward"] == n0
        # unrelated eager work between replays (library and torch)
        x = (m0 * 2.0).sum()
        c.forward(shot, m0, q)
        torch.cuda.synchronize()
        assert torch.isfinite(x)
    # a call on another grid reallocates the fields: the next call re-captures
    c.forward(other, om, oq)
    phi, _ = c.gradient(shot, m0, q, d, nslots=4, compress=compress, atol=1e-4, grad=g)
    assert torch.equal(g, g0) and phi == phi0
    c.set_graphs(False)
    phi, g2 = c.gradient(shot, m0, q, d, nslots=4, compress=compress, atol=1e-4)
    assert torch.equal(g2, g0)
    c.close()


@pytest.mark.parametrize("compress", [True, False])
def test_graph_replays_equal_direct_batched(compress):
    c = F.Context(0, pool_bytes=1 << 28)
    probs = [problem(3, n, 8, nt=40, seed=s) for n, s in ((16, 1), (21, 2), (18, 3))]
    shots = [p[0] for p in probs]
    m0s = [p[1] for p in probs]
    q = probs[0][3]
    dobs = [c.forward(s, mt, q) for s, _, mt, _ in probs]
    phis0, g0 = c.gradient_batch(shots, m0s, q, dobs, nslots=3, compress=compress, atol=1e-4)
    c.set_graphs(True)
    gs = [torch.empty_like(m) for m in m0s]
    for i in range(3):
        for g in gs:
            g.fill_(float("nan"))
        phis, _ = c.gradient_batch(shots, m0s, q, dobs, nslots=3, compress=compress, atol=1e-4,
                                   grads=gs)
        for a, b in zip(gs, g0):
            assert torch.equal(a, b), i
        assert phis == phis0
        c.gradient(shots[0], m0s[0], q, dobs[0], nslots=2)
        torch.cuda.synchronize()
    c.close()


def test_graph_on_a_user_stream():
    c = F.Context(0, pool_bytes=1 << 27)
    shot, m0, mt, q = problem(2, 40, 8, nt=40)
    d = c.forward(shot, mt, q)
    phi0, g0 = c.gradient(shot, m0, q, d, nslots=3, compress=True, atol=1e-4)
    c.set_graphs(True)
    s = torch.cuda.Stream()
    g = torch.empty_like(m0)
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(3):
            phi, _ = c.gradient(shot, m0, q, d, nslots=3, compress=True, atol=1e-4, grad=g)
    s.synchronize()
    assert torch.equal(g, g0) and phi == phi0
    c.close()


@pytest.mark.parametrize("ndim,compress", [(2, True), (3, False), (3, True)])
def test_tape_graphs_replay_equal_direct(ndim, compress):
    """the split (autograd) form: forward tape and backward captured once,
    then replayed with the tape buffers the context keeps from the freed
    tape, equal bit for bit to direct launches every time"""
    c = F.Context(0, pool_bytes=1 << 27)
    shot, m0, mt, q = problem(ndim, 40 if ndim == 2 else 16, 8, nt=40)
    d_obs = c.forward(shot, mt, q)
    d0, tape = c.forward_ckpt(shot, m0, q, nslots=4, compress=compress, atol=1e-4, pool_bytes=1 << 25)
    dd = (d0 - d_obs).contiguous()
    g0 = c.backward(tape, dd)
    tape.free()
    c.set_graphs(True)
    d, g = torch.empty_like(d0), torch.empty_like(m0)
    for i in range(4):
        d.fill_(float("nan"))
        g.fill_(float("nan"))
        _, tape = c.forward_ckpt(shot, m0, q, nslots=4, compress=compress, atol=1e-4, pool_bytes=1 << 25,
                                 d_sim=d)
        sf = c.stats()
        c.backward(tape, dd, grad=g)
        sb = c.stats()
        tape.free()
        assert torch.equal(d, d0) and torch.equal(g, g0), i
        if i > 0:
            assert sf["graphs_replayed"] == 1 and sb["graphs_replayed"] == 1, (i, sf, sb)
        c.forward(shot, mt, q)           # eager work between replays
        torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("compress", [True, False])
def test_batched_tape_graphs_replay_equal_direct(compress):
    """the batched autograd op's calls (forward tape, stacked backward) with
    graphs on: replays equal direct launches bit for bit"""
    c = F.Context(0, pool_bytes=1 << 28)
    base, m0, mt, q = problem(2, 44, 8, nt=40)
    shots = []
    for x in (6, 20, 37):
        s = synth.Shot(2, base.shape, base.h, base.so, base.nbl, base.nt, base.dt, base.vmax, base.f0,
                       (x, 2), base.rec)
        shots.append(s)
    d_obs = [c.forward(s, mt, q) for s in shots]
    ref_ds, tape = c.forward_ckpt_batch(shots, [m0] * 3, q, nslots=4, compress=compress, atol=1e-4,
                                        pool_bytes=1 << 26)
    dds = [(a - b).contiguous() for a, b in zip(ref_ds, d_obs)]
    dims = tuple(m0.shape)
    g0 = c.backward_stack(tape, dds, dims, 0, [(0, 0)] * 3)
    tape.free()
    c.set_graphs(True)
    ds = [torch.empty_like(x) for x in ref_ds]
    g = torch.empty_like(m0)
    for i in range(3):
        for x in ds:
            x.fill_(float("nan"))
        g.fill_(float("nan"))
        _, tape = c.forward_ckpt_batch(shots, [m0] * 3, q, nslots=4, compress=compress, atol=1e-4,
                                       pool_bytes=1 << 26, d_sim=ds)
        sf = c.stats()
        c.backward_stack(tape, dds, dims, 0, [(0, 0)] * 3, grad=g)
        sb = c.stats()
        tape.free()
        for a, b in zip(ds, ref_ds):
            assert torch.equal(a, b), i
        assert torch.equal(g, g0), i
        if i > 0:
            assert sf["graphs_replayed"] == 1 and sb["graphs_replayed"] == 1, (i, sf, sb)
        torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("batched", [False, True])
def test_autograd_graphs_replay_with_fresh_tensors(batched):
    """autograd iterations allocate new model, trace, residual and gradient
    tensors every time; captured tape schedules still replay (the graphs
    read and write only context and tape buffers, with copies in and out
    around each replay) and equal the direct launches bit for bit"""
    c = F.Context(0, pool_bytes=1 << 28)
    base, m0, mt, q = problem(2, 44, 8, nt=40)
    shots = [synth.Shot(2, base.shape, base.h, base.so, base.nbl, base.nt, base.dt, base.vmax, base.f0,
                        (x, 2), base.rec) for x in (6, 20, 37)]
    d_obs = [c.forward(s, mt, q) for s in shots]

    def iteration():
        m = m0.clone().requires_grad_(True)
        if batched:
            ds = F.forward_modelling_batch(c, m, shots, q, nslots=4, compress=True, atol=1e-4,
                                           pool_bytes=1 << 26)
            sf = c.stats()
        else:
            op = F.FwiOperator(c, nslots=4, compress=True, atol=1e-4)
            ds = [op(m, s, q) for s in shots]
            sf = c.stats()
        loss = sum(0.5 * ((d - o) ** 2).sum() for d, o in zip(ds, d_obs))
        loss.backward()
        return [d.detach().clone() for d in ds], m.grad.clone(), sf, c.stats()

    ref_d, ref_g, _, _ = iteration()
    c.set_graphs(True)
    keep = []
    for i in range(4):
        ds, g, sf, sb = iteration()
        keep.append(torch.empty(1000 + 17 * i, device=DEV))   # moves torch's next allocations
        for a, b in zip(ds, ref_d):
            assert torch.equal(a, b), i
        assert torch.equal(g, ref_g), i
        if i > 0:
            assert sf["graphs_replayed"] == 1 and sb["graphs_replayed"] == 1, (i, sf, sb)
        torch.cuda.synchronize()
    c.set_graphs(False)
    c.close()


@pytest.mark.parametrize("batched", [False, True])
def test_gradient_graphs_replay_with_fresh_buffers(batched):
    """fwi_gradient / fwi_gradient_batch with new model, observed-data and
    gradient tensors every call: the captured schedule replays (it reads the
    context's copy of the data and stops at the padded accumulators) and
    equals direct launches bit for bit"""
    c = F.Context(0, pool_bytes=1 << 28)
    probs = [problem(3, n, 8, nt=40, seed=s) for n, s in ((16, 1), (21, 2))]
    shots = [p[0] for p in probs]
    q = probs[0][3]
    dobs = [c.forward(s, mt, q) for s, _, mt, _ in probs]

    def call(fresh):
        m0s = [p[1].clone() if fresh else p[1] for p in probs]
        ds = [d.clone() if fresh else d for d in dobs]
        if batched:
            gs = [torch.full_like(m, float("nan")) for m in m0s]
            phis, _ = c.gradient_batch(shots, m0s, q, ds, nslots=3, compress=True, atol=1e-4, grads=gs)
            return phis, gs
        g = torch.full_like(m0s[0], float("nan"))
        phi, _ = c.gradient(shots[0], m0s[0], q, ds[0], nslots=3, compress=True, atol=1e-4, grad=g)
        return [phi], [g]

    phis0, g0 = call(False)
    c.set_graphs(True)
    keep = []
    for i in range(3):
        phis, gs = call(True)
        keep.append(torch.empty(333 + 29 * i, device=DEV))
        assert phis == phis0, i
        for a, b in zip(gs, g0):
            assert torch.equal(a, b), i
        if i > 0:
            assert c.stats()["graphs_replayed"] == 1, i
        torch.cuda.synchronize()
    c.close()
