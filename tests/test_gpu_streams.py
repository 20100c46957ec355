"""The checkpoint streams a compressed tape actually stores (paper Sec. 1.3
checkpointing with Sec. 1.4 compression: each stored level is the codec
stream of the forward state at the checkpoint's step), byte for byte against
the oracle's compression of the same float32 state.  The states come from
fwi_forward_span (chained spans equal one sweep bit for bit), so this pins
the pool-placement encode path (streams placed on the device-side stack)
rather than the dense-destination path ckpt_compress uses."""
import numpy as np
import pytest
import torch

import synth
from oracle import codec as ocodec

pytestmark = pytest.mark.gpu
F = pytest.importorskip("paper_2009_12623_amd.fwigrad")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def inputs(shot, seed=3):
    v0, vt = synth.tiny_models(shot.shape, seed=seed)
    m0 = synth.slowness2(synth.extend(v0, shot.nbl)).astype(np.float32)
    q = shot.wavelet().astype(np.float32)
    return m0, q


def first_sweep_checkpoints(nt, nslots):
    """(slot, step, holds u^(k-1)) of every takeshot before the first
    reverse step; a checkpoint keeps the older level only when the schedule
    later restores it and advances from it"""
    acts, _ = F.fwi_revolve_plan(nt, nslots)
    shots, last = [], {}
    for i, a in enumerate(acts):
        if a[0] == "takeshot":
            last[a[1]] = i
    for i, a in enumerate(acts):
        if a[0] == "reverse":
            break
        if a[0] == "takeshot":
            shots.append((a[1], a[2], i))
    out = []
    for slot, k, i in shots:
        both = False
        for j in range(i + 1, len(acts) - 1):
            if acts[j][0] == "takeshot" and acts[j][1] == slot:
                break
            if acts[j][0] == "restore" and acts[j][1] == slot and acts[j + 1][0] == "advance":
                both = True
                break
        out.append((slot, k, both))
    return out


def gpu_states(ctx, shot, m, q, k):
    """(u^k, u^(k-1)) of the GPU's own sweep, unpadded float32"""
    u = torch.zeros(m.shape, dtype=torch.float32, device="cuda:0")
    v = torch.zeros_like(u)
    ctx.forward_span(shot, m, q, 0, k, u, v)
    return u.cpu().numpy(), v.cpu().numpy()


@pytest.mark.parametrize("ndim,n,so,nt,nslots,atol,waves", [
    (2, 60, 8, 40, 40, 1e-4, 0),       # store-all: every step a checkpoint
    (2, 60, 16, 50, 4, 1e-3, 0),       # recomputing: some checkpoints hold both levels
    (3, 22, 8, 24, 24, 1e-4, 0),
    (3, 22, 4, 30, 3, 1e-2, 0),
    (3, 22, 8, 24, 24, 1e-4, 1),       # codec launches capped at 1 or 3 waves, each looping
    (3, 22, 4, 30, 3, 1e-2, 3),        # over the chunk groups: same streams
])
def test_tape_streams_equal_oracle_compression(ndim, n, so, nt, nslots, atol, waves, monkeypatch):
    if waves:
        monkeypatch.setenv("FWI_CODEC_WAVES", str(waves))
    ctx = F.Context(0, pool_bytes=1 << 27)
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=5, nt=nt)
    m0, q = inputs(shot)
    m, qd = dev(m0), dev(q)
    _, tape = ctx.forward_ckpt(shot, m, qd, nslots=nslots, compress=True, atol=atol,
                               pool_bytes=1 << 26)
    cks = first_sweep_checkpoints(nt, nslots)
    assert cks and any(k > 0 for _, k, _ in cks)
    nboth = 0
    for slot, k, both in cks:
        uk, ukm1 = gpu_states(ctx, shot, m, qd, k)
        got = tape.stream(slot, 0).cpu().numpy().tobytes()
        assert got == ocodec.compress(uk, atol), (slot, k)
        if both:
            nboth += 1
            got1 = tape.stream(slot, 1).cpu().numpy().tobytes()
            assert got1 == ocodec.compress(ukm1, atol), (slot, k)
        else:
            with pytest.raises(F.FwiError):
                tape.stream(slot, 1)
    if nslots < nt:
        assert nboth > 0
    tape.free()
    ctx.close()


def test_batched_tape_streams_equal_oracle_compression():
    """uneven shots in one batched tape: each shot's stored streams"""
    ctx = F.Context(0, pool_bytes=1 << 27)
    nt, nslots, atol = 30, 4, 1e-4
    shots = [synth.tiny_shot(2, n=n, so=8, nbl=5, nt=nt) for n in (40, 57)]
    ms, qs = [], []
    for s in shots:
        m0, q = inputs(s)
        ms.append(dev(m0))
        qs.append(dev(q))
    _, tape = ctx.forward_ckpt_batch(shots, ms, qs[0], nslots=nslots, compress=True, atol=atol,
                                     pool_bytes=1 << 26)
    cks = first_sweep_checkpoints(nt, nslots)
    for i, s in enumerate(shots):
        for slot, k, both in cks:
            uk, ukm1 = gpu_states(ctx, s, ms[i], qs[0], k)
            assert tape.stream(slot, 0, shot=i).cpu().numpy().tobytes() == ocodec.compress(uk, atol)
            if both:
                assert tape.stream(slot, 1, shot=i).cpu().numpy().tobytes() == ocodec.compress(ukm1, atol)
    tape.free()
    ctx.close()


def test_exact_tape_has_no_streams():
    ctx = F.Context(0, pool_bytes=1 << 26)
    shot = synth.tiny_shot(2, n=30, so=4, nbl=4, nt=20)
    m0, q = inputs(shot)
    _, tape = ctx.forward_ckpt(shot, dev(m0), dev(q), nslots=4, compress=False, pool_bytes=1 << 25)
    with pytest.raises(F.FwiError) as e:
        tape.stream(0, 0)
    assert e.value.code == F.FWI_EINVAL
    tape.free()
    ctx.close()
