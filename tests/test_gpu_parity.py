"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: FP32 receiver traces and gradients within relative L2 1e-4 of the FP64
oracle; compressed streams bit-exact; uncompressed checkpointing bitwise equal
to store-all (paper Sec. 1.3); compressed-checkpoint gradient within relative
L2 1e-3 of the uncompressed one.  Sizes span several stencil tiles and codec
chunks with ragged tails.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import codec as ocodec
from oracle import metrics, solver

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_2009_12623_amd.fwigrad")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = F.Context(0, pool_bytes=1 << 30)
    yield c
    c.close()


def inputs(shot, seed=3):
    v0, vt = synth.tiny_models(shot.shape, seed=seed)
    m0 = synth.slowness2(synth.extend(v0, shot.nbl)).astype(np.float32)
    mt = synth.slowness2(synth.extend(vt, shot.nbl)).astype(np.float32)
    q = shot.wavelet().astype(np.float32)
    return m0, mt, q


def oracle_problem(shot, m32, q32):
    return solver.Problem(shot, m32.astype(np.float64), wavelet=q32.astype(np.float64))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


CASES = [
    # ndim, n, so, nbl, nt
    (2, 37, 4, 6, 60),
    (2, 70, 16, 10, 80),
    (2, 300, 8, 8, 120),     # two 2D z-tiles, ragged
    (3, 19, 8, 5, 40),
    (3, 26, 4, 4, 30),       # several y tiles, ragged
    (3, 14, 16, 4, 30),
]


@pytest.mark.parametrize("ndim,n,so,nbl,nt", CASES)
def test_forward_traces_match_oracle(ctx, ndim, n, so, nbl, nt):
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=nbl, nt=nt)
    m0, _, q = inputs(shot)
    d = ctx.forward(shot, dev(m0), dev(q)).cpu().numpy()
    dref = solver.forward(oracle_problem(shot, m0, q))
    err = metrics.rel_l2(d, dref)
    print("forward", ndim, n, so, "rel L2 vs FP64", err)
    assert err <= 1e-4


@pytest.mark.parametrize("ndim,n,so,nbl,nt", CASES)
def test_gradient_matches_oracle(ctx, ndim, n, so, nbl, nt):
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=nbl, nt=nt)
    m0, mt, q = inputs(shot)
    p0 = oracle_problem(shot, m0, q)
    pt = oracle_problem(shot, mt, q)
    dobs = solver.forward(pt)
    phi_ref, gref, _ = solver.gradient(p0, dobs)
    phi, g = ctx.gradient(shot, dev(m0), dev(q), dev(dobs.astype(np.float32)), nslots=nt)
    g = g.cpu().numpy()
    err = metrics.rel_l2(g, gref)
    print("gradient", ndim, n, so, "rel L2 vs FP64", err, "phi", phi, phi_ref)
    assert err <= 1e-4
    assert abs(phi - phi_ref) <= 1e-4 * phi_ref


@pytest.mark.parametrize("ndim,n,so", [(2, 60, 16), (3, 22, 8)])
def test_forward_state_matches_oracle(ctx, ndim, n, so):
    """the last two levels returned by fwi_forward_state"""
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=5, nt=50)
    m0, _, q = inputs(shot)
    d, u1, u0 = ctx.forward_state(shot, dev(m0), dev(q))
    dref, states = solver.forward(oracle_problem(shot, m0, q), keep_states=True)
    assert metrics.rel_l2(d.cpu().numpy(), dref) <= 1e-4
    assert metrics.rel_l2(u1.cpu().numpy(), states[shot.nt]) <= 1e-4
    assert metrics.rel_l2(u0.cpu().numpy(), states[shot.nt - 1]) <= 1e-4


def _deep_shot(so, zsrc, nt=30):
    """3D shot whose computational depth (281) spans three 128-point z tiles
    with an odd tail and whose y extent (31) leaves a ragged tile; source and
    receivers at physical depth zsrc (123: across the first tile boundary,
    268: in the tail tile), so both sweeps run there"""
    shape, nbl = (18, 21, 271), 5
    dt = synth.stable_dt(10.0, 2500.0, 3, so, 0.8)
    ix, iy = np.meshgrid(np.arange(0, 18, 3), np.arange(0, 21, 4), indexing="ij")
    rz = np.clip(zsrc + (ix + iy) % 7 - 3, 0, 270)
    rec = np.stack([ix.ravel(), iy.ravel(), rz.ravel()], 1).astype(np.int32)
    return synth.Shot(3, shape, 10.0, so, nbl, nt, dt, 2500.0, 1500.0 / 80.0, (9, 10, zsrc), rec)


_SHAPES = [(3, 2, 0, 0, 1), (7, 4, 1, 0, 1), (64, 2, 1, 0, 1), (16, 4, 0, 0, 1), (16, 2, 2, 0, 1),
           (7, 4, 2, 0, 1), (5, 2, 2, 1, 1), (3, 2, 0, 1, 1), (16, 2, 1, 1, 1), (64, 2, 0, 1, 1),
           (1, 2, 0, 1, 1), (2, 2, 0, 1, 1), (3, 2, 0, 0, 2), (7, 4, 1, 0, 2), (16, 2, 2, 0, 2),
           (64, 4, 2, 0, 2), (1, 4, 0, 0, 2), (5, 2, 1, 0, 2), (16, 2, 3, 0, 1), (7, 2, 4, 0, 1),
           (3, 4, 4, 0, 1), (5, 2, 3, 0, 2)]
# every shape on the cube grid at SO 4/8/16; the deep grids (several z tiles,
# ragged tail) with SO 8/16 for the two-point lanes and three one-point shapes
_SHAPE_CASES = [sh + (so, grid) for grid in ("cube", "deep_mid", "deep_tail") for so in (4, 8, 16)
                for sh in _SHAPES
                if grid == "cube" or (so != 4 and (sh[4] == 2 or (sh[0], sh[1]) in ((16, 2), (7, 4), (7, 2))))]


@pytest.mark.parametrize("xchunk,rpl,remap,deep,vz,so,grid", _SHAPE_CASES)
def test_3d_stencil_launch_shapes_match_oracle(xchunk, rpl, remap, deep, vz, so, grid, monkeypatch):
    """every launch shape (x planes per workgroup, rows per lane, tile order,
    loads of one or two planes in flight, one or two z points per lane); the
    deep grids span several 128-point z tiles with a ragged, odd tail"""
    monkeypatch.setenv("FWI_XCHUNK", str(xchunk))
    monkeypatch.setenv("FWI_RPL", str(rpl))
    monkeypatch.setenv("FWI_REMAP", str(remap))
    monkeypatch.setenv("FWI_DEEP", str(deep))
    monkeypatch.setenv("FWI_VZ", str(vz))
    c = F.Context(0, pool_bytes=1 << 28)
    shot = (synth.tiny_shot(3, n=23, so=so, nbl=5, nt=35) if grid == "cube"
            else _deep_shot(so, 123 if grid == "deep_mid" else 268))
    m0, mt, q = inputs(shot)
    p0 = oracle_problem(shot, m0, q)
    dobs = solver.forward(oracle_problem(shot, mt, q))
    phi_ref, gref, dref = solver.gradient(p0, dobs)
    d = c.forward(shot, dev(m0), dev(q)).cpu().numpy()
    assert metrics.rel_l2(d, dref) <= 1e-4
    phi, g = c.gradient(shot, dev(m0), dev(q), dev(dobs.astype(np.float32)), nslots=3)
    assert metrics.rel_l2(g.cpu().numpy(), gref) <= 1e-4
    c.close()


@pytest.mark.parametrize("xchunk", [1, 3, 4, 7, 16, 64])
@pytest.mark.parametrize("so", [4, 8, 16])
def test_2d_stencil_launch_shapes_match_oracle(xchunk, so, monkeypatch):
    """2D launch shapes (x planes per workgroup) on a grid of two 256-point
    z tiles with a ragged tail and x chunks that do not divide it: traces
    and gradient against the oracle"""
    monkeypatch.setenv("FWI_XCHUNK", str(xchunk))
    shot = synth.tiny_shot(2, n=290, so=so, nbl=5, nt=35)
    m0, mt, q = inputs(shot)
    p0 = oracle_problem(shot, m0, q)
    dobs = solver.forward(oracle_problem(shot, mt, q))
    _, gref, dref = solver.gradient(p0, dobs)
    c = F.Context(0, pool_bytes=1 << 27)
    d = c.forward(shot, dev(m0), dev(q)).cpu().numpy()
    _, g = c.gradient(shot, dev(m0), dev(q), dev(dobs.astype(np.float32)), nslots=3)
    c.close()
    assert metrics.rel_l2(d, dref) <= 1e-4
    assert metrics.rel_l2(g.cpu().numpy(), gref) <= 1e-4


@pytest.mark.parametrize("xchunk,rpl,remap,vz", [(16, 2, 2, 1), (7, 4, 0, 1), (3, 2, 0, 2), (7, 4, 1, 2),
                                                 (16, 2, 2, 2), (64, 4, 2, 2), (1, 4, 0, 2), (16, 2, 3, 1),
                                                 (3, 2, 4, 1), (7, 4, 4, 2)])
@pytest.mark.parametrize("so", [8, 16])
def test_forward_steps_from_random_states_every_tile(xchunk, rpl, remap, vz, so, monkeypatch):
    """three forward steps from seeded random states on the deep grid: every
    z tile, the odd z tail and the ragged y tile hold data, against the
    oracle's steps on every point"""
    monkeypatch.setenv("FWI_XCHUNK", str(xchunk))
    monkeypatch.setenv("FWI_RPL", str(rpl))
    monkeypatch.setenv("FWI_REMAP", str(remap))
    monkeypatch.setenv("FWI_VZ", str(vz))
    c = F.Context(0, pool_bytes=1 << 26)
    shot = _deep_shot(so, 123, nt=8)
    m0, _, q = inputs(shot)
    rng = np.random.default_rng(21)
    u1 = rng.standard_normal(shot.comp_shape).astype(np.float32)
    u0 = rng.standard_normal(shot.comp_shape).astype(np.float32)
    p = oracle_problem(shot, m0, q)
    cur, prev = u1.astype(np.float64), u0.astype(np.float64)
    for k in range(3, 6):
        cur, prev = p.step(cur, prev, [p.src], [p.q[k]]), cur
    g1, g0 = dev(u1), dev(u0)
    c.forward_span(shot, dev(m0), dev(q), 3, 6, g1, g0)
    assert metrics.rel_l2(g1.cpu().numpy(), cur) <= 1e-5
    assert metrics.rel_l2(g0.cpu().numpy(), prev) <= 1e-5
    c.close()


@pytest.mark.parametrize("ndim,n,so", [(2, 150, 16), (3, 40, 8)])
def test_autotuned_shapes_keep_the_gradient(ndim, n, so):
    """the autotuner picks a listed shape; the gradient it then computes
    equals the oracle's like the default shape's does"""
    c = F.Context(0, pool_bytes=1 << 28)
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=6, nt=40)
    m0, mt, q = inputs(shot)
    p0 = oracle_problem(shot, m0, q)
    dobs = solver.forward(oracle_problem(shot, mt, q))
    _, gref, _ = solver.gradient(p0, dobs)
    _, g_def = c.gradient(shot, dev(m0), dev(q), dev(dobs.astype(np.float32)), nslots=4)
    r = c.autotune(shot, dev(m0), dev(q), steps=2)
    print("autotune", ndim, r)
    assert r["ncand"] == (63 if ndim == 3 else 5)
    assert r["fwd_xchunk"] in (4, 8, 16, 32, 64) and r["adj_xchunk"] in (4, 8, 16, 32, 64)
    assert r["fwd_rows_per_lane"] in (2, 4) and r["fwd_ms"] > 0 and r["adj_ms"] > 0
    _, g = c.gradient(shot, dev(m0), dev(q), dev(dobs.astype(np.float32)), nslots=4)
    g, g_def = g.cpu().numpy(), g_def.cpu().numpy()
    assert metrics.rel_l2(g, gref) <= 1e-4
    assert metrics.rel_l2(g, g_def) <= 1e-6
    c.close()


@pytest.mark.parametrize("nslots", [0, 1, 3, 7])
@pytest.mark.parametrize("ndim", [2, 3])
def test_revolve_is_bitwise_store_all(ctx, ndim, nslots):
    shot = synth.tiny_shot(ndim, n=30 if ndim == 2 else 16, so=8, nbl=5, nt=45)
    m0, mt, q = inputs(shot)
    dobs = ctx.forward(shot, dev(mt), dev(q))
    phi_a, ga = ctx.gradient(shot, dev(m0), dev(q), dobs, nslots=shot.nt)
    phi_b, gb = ctx.gradient(shot, dev(m0), dev(q), dobs, nslots=nslots)
    assert phi_a == phi_b
    assert torch.equal(ga, gb)
    st = ctx.stats()
    from oracle import revolve
    assert st["n_forward"] == revolve.T_closed(shot.nt, min(nslots, shot.nt))
    assert st["n_adjoint"] == shot.nt


@pytest.mark.parametrize("ndim,so", [(2, 4), (3, 8)])
def test_compressed_gradient_close_to_exact(ctx, ndim, so):
    shot = synth.tiny_shot(ndim, n=48 if ndim == 2 else 20, so=so, nbl=6, nt=70)
    m0, mt, q = inputs(shot)
    dobs = ctx.forward(shot, dev(mt), dev(q))
    _, gexact = ctx.gradient(shot, dev(m0), dev(q), dobs, nslots=5)
    errs = []
    for atol in (1e-2, 1e-4, 1e-5):
        _, gc = ctx.gradient(shot, dev(m0), dev(q), dobs, nslots=5, compress=True, atol=atol)
        errs.append(metrics.rel_l2(gc.cpu().numpy(), gexact.cpu().numpy()))
        st = ctx.stats()
        assert st["n_encode"] > 0 and st["n_decode"] > 0
    print("compressed gradient rel errors", errs)
    assert errs[1] <= 1e-3
    assert errs[2] <= errs[0]


@pytest.mark.parametrize("ndim,n,so,nt,nslots", [(2, 40, 4, 60, 4), (2, 90, 16, 160, 6),
                                                (3, 24, 8, 90, 5), (3, 20, 16, 100, 100)])
def test_compressed_gradient_matches_oracle_compressed(ctx, ndim, n, so, nt, nslots):
    """lossy GPU gradient (atol 1e-4) against the oracle's lossy gradient
    (FP64 states rounded to float32 and compressed, Sec. 3) at the same bar
    as the exact gradient; each side compresses its own states, so the
    streams may differ where a value sits on a quantisation boundary"""
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=6, nt=nt)
    v0, vt = synth.tiny_models(shot.shape, seed=3)
    vt = v0 * (1.0 + 4.0 * (vt / v0 - 1.0))          # a residual of several % of the data
    m0 = synth.slowness2(synth.extend(v0, shot.nbl)).astype(np.float32)
    mt = synth.slowness2(synth.extend(vt, shot.nbl)).astype(np.float32)
    q = shot.wavelet().astype(np.float32)
    p0 = oracle_problem(shot, m0, q)
    dobs = solver.forward(oracle_problem(shot, mt, q))
    st = {}
    _, gref = solver.gradient_checkpointed(p0, dobs, nslots, atol=1e-4, stats=st)
    rr = np.linalg.norm(st["d_sim"] - dobs) / np.linalg.norm(dobs)
    _, g = ctx.gradient(shot, dev(m0), dev(q), dev(dobs.astype(np.float32)), nslots=nslots,
                        compress=True, atol=1e-4)
    err = metrics.rel_l2(g.cpu().numpy(), gref)
    print("lossy vs lossy oracle", ndim, so, "residual/data %.3f" % rr, "err %.2e" % err)
    assert rr >= 0.02
    assert err <= 1e-4


def test_autograd_split_equals_gradient(ctx):
    shot = synth.tiny_shot(2, n=33, so=8, nbl=5, nt=50)
    m0, mt, q = inputs(shot)
    dobs = ctx.forward(shot, dev(mt), dev(q))
    for compress in (False, True):
        phi, g = ctx.gradient(shot, dev(m0), dev(q), dobs, nslots=4, compress=compress, atol=1e-4)
        d, tape = ctx.forward_ckpt(shot, dev(m0), dev(q), nslots=4, compress=compress, atol=1e-4,
                                   pool_bytes=1 << 26)
        g2 = ctx.backward(tape, d - dobs)
        tape.free()
        assert torch.equal(g, g2)


# ------------------------------------------------------------------ codec
def codec_fields():
    rng = np.random.default_rng(21)
    yield synth.wavefield_like((37, 29, 45), seed=1)
    yield synth.wavefield_like((130, 97), seed=2)
    yield synth.wavefield_like((64, 64, 64), seed=3, noise=1e-3)
    yield (rng.standard_normal((9, 17, 70)) * 3).astype(np.float32)
    yield np.zeros((5, 6, 7), np.float32)
    yield np.full((3, 2), 1.5, np.float32)
    yield (rng.standard_normal((1, 1)) * 1.0).astype(np.float32)
    x = (rng.standard_normal((33, 65)) * 2.0 ** rng.integers(-20, 6, (33, 65))).astype(np.float32)
    x[0, :5] = np.float32(1e-42)         # subnormals count as zero
    yield x
    # tiny magnitudes: at the smallest atol reconstructions below 2^-126
    # flush to +0
    yield (rng.standard_normal((12, 9, 11)) * 1e-37).astype(np.float32)


@pytest.mark.parametrize("atol", [1e-1, 1e-3, 1e-4, 1e-6, 2.0 ** -70, 2.0 ** -140])
def test_codec_streams_bit_exact(ctx, atol):
    """streams and decodes byte-identical to the oracle's; where the oracle
    refuses a field (a value at or above atol 2^23) the library refuses it
    too, with FWI_ERANGE"""
    for x in codec_fields():
        try:
            ref = ocodec.compress(x, atol)
        except ocodec.CodecError as e:
            assert e.code == ocodec.ERANGE
            with pytest.raises(F.FwiError) as ge:
                ctx.compress(dev(x), atol)
            assert ge.value.code == F.FWI_ERANGE
            continue
        s = ctx.compress(dev(x), atol).cpu().numpy().tobytes()
        assert s == ref, (x.shape, atol, len(s), len(ref))
        y = ctx.decompress(dev(np.frombuffer(ref, np.uint8).copy()), x.shape).cpu().numpy()
        yref = ocodec.decompress(ref, x.shape)
        assert np.array_equal(y.view(np.uint32), yref.view(np.uint32))


def test_codec_saturation_bit_exact(ctx):
    """values at the top of float32 whose reconstructions exceed the largest
    float (they saturate to it): the oracle's stream and decode, bit for bit"""
    rng = np.random.default_rng(22)
    x = (rng.uniform(3.4e38, 3.4028234e38, (10, 13)) * rng.choice([-1.0, 1.0], (10, 13))).astype(np.float32)
    with pytest.raises(F.FwiError) as e:            # far beyond atol 2^23
        ctx.compress(dev(x), 1e-1)
    assert e.value.code == F.FWI_ERANGE
    for atol in (1e36, 2.0 ** 105):
        ref = ocodec.compress(x, atol)
        assert ctx.compress(dev(x), atol).cpu().numpy().tobytes() == ref
        y = ctx.decompress(dev(np.frombuffer(ref, np.uint8).copy()), x.shape).cpu().numpy()
        yref = ocodec.decompress(ref, x.shape)
        assert np.array_equal(y.view(np.uint32), yref.view(np.uint32))
        if atol == 1e36:
            assert np.sum(np.abs(yref) == np.float32(3.4028235e38)) > 0    # the case is exercised


@pytest.mark.parametrize("shape,kblk", [((100, 100, 100), 1), ((200, 200, 200), 4),
                                        ((256, 256, 256), 16), ((1081, 481), 2),
                                        ((4100, 4100), 64)])
def test_codec_chunk_lengths_bit_exact(ctx, shape, kblk):
    """fields whose size selects each chunk length K (blocks per chunk, from
    the block count), up to the 256^3 snapshot size; streams byte-identical
    to the oracle's and decodes bit-identical"""
    x = synth.wavefield_like(shape, seed=7)
    ref = ocodec.compress(x, 1e-4)
    h = ocodec.header(ref)
    nblocks = int(np.prod([(n + 3) // 4 for n in shape]))
    assert h["nchunks"] == 64 * -(-nblocks // (64 * kblk))
    s = ctx.compress(dev(x), 1e-4).cpu().numpy().tobytes()
    assert s == ref
    y = ctx.decompress(dev(np.frombuffer(ref, np.uint8).copy()), shape).cpu().numpy()
    assert np.array_equal(y.view(np.uint32), ocodec.decompress(ref, shape).view(np.uint32))


def padded_array(x, pad=8):
    """x inside a zero array with `pad` points before and after every axis
    and 16-byte aligned rows: (array, origin offset, sx, sy)"""
    if x.ndim == 3:
        n0, n1, n2 = x.shape
        pz = (2 * pad + n2 + 3) // 4 * 4
        a = np.zeros((n0 + 2 * pad, n1 + 2 * pad, pz), np.float32)
        a[pad:pad + n0, pad:pad + n1, pad:pad + n2] = x
        sy, sx = pz, (n1 + 2 * pad) * pz
        return a, pad * sx + pad * sy + pad, sx, sy
    n0, n2 = x.shape
    pz = (2 * pad + n2 + 3) // 4 * 4
    a = np.zeros((n0 + 2 * pad, pz), np.float32)
    a[pad:pad + n0, pad:pad + n2] = x
    return a, pad * pz + pad, pz, 0


@pytest.mark.parametrize("shape", [(37, 29, 45), (70, 66, 367), (130, 97), (181, 181)])
@pytest.mark.parametrize("atol", [1e-3, 1e-5])
def test_codec_views_bit_exact(ctx, shape, atol):
    """the codec on a field inside a larger array (the layout checkpoints
    use, padded = whole-block access): the same stream as the dense field,
    and a padded decode writes the values and leaves every pad point zero"""
    x = synth.wavefield_like(shape, seed=11)
    ref = ocodec.compress(x, atol)
    a, off, sx, sy = padded_array(x)
    A = dev(a)
    for padded in (True, False):
        s = ctx.compress_view(A, off, shape, sx, sy, padded, atol).cpu().numpy().tobytes()
        assert s == ref, padded
    yref = ocodec.decompress(ref, shape)
    for padded in (True, False):
        Q = torch.zeros_like(A)
        ctx.decompress_view(dev(np.frombuffer(ref, np.uint8).copy()), Q, off, shape, sx, sy, padded)
        q = Q.cpu().numpy()
        inner = tuple(slice(8, 8 + n) for n in shape)
        assert np.array_equal(q[inner].view(np.uint32), yref.view(np.uint32)), padded
        q[inner] = 0.0
        assert not q.any(), padded


def test_codec_view_rejects_bad_layouts(ctx):
    x = synth.wavefield_like((20, 20, 20), seed=2)
    a, off, sx, sy = padded_array(x)
    A = dev(a)
    with pytest.raises(F.FwiError):
        ctx.compress_view(A, off + 1, x.shape, sx, sy, True, 1e-3)      # misaligned rows
    with pytest.raises(F.FwiError):
        ctx.compress_view(A, off, x.shape, sx, 19, False, 1e-3)         # rows overlap
    s = ctx.compress_view(A, off + 1, x.shape, sx, sy, False, 1e-3)     # fine unpadded
    assert s.numel() > 64


def test_codec_on_oracle_wavefields(ctx):
    # float32-rounded states of an oracle FP64 propagation (2D and 3D)
    for ndim, n in ((2, 90), (3, 30)):
        shot = synth.tiny_shot(ndim, n=n, so=8, nbl=6, nt=60)
        m0, _, q = inputs(shot)
        _, states = solver.forward(oracle_problem(shot, m0, q), keep_states=True)
        for k in (10, 35, 60):
            x = states[k].astype(np.float32)
            for atol in (1e-2, 1e-4):
                ref = ocodec.compress(x, atol)
                s = ctx.compress(dev(x), atol).cpu().numpy().tobytes()
                assert s == ref


@pytest.mark.parametrize("ndim", [2, 3])
def test_codec_refuses_values_beyond_the_accuracy_range(ctx, ndim):
    """|x - x_hat| <= atol needs every |x| below 2^(floor(log2 atol) + 23):
    just below the limit the stream is the oracle's and the bound holds; at
    it the library returns FWI_ERANGE, also from a compressed gradient"""
    atol = 2.0 ** -20
    shape = (9, 6, 7) if ndim == 3 else (13, 10)
    rng = np.random.default_rng(31)
    x = rng.uniform(-1, 1, shape).astype(np.float32)
    x.flat[17] = np.nextafter(np.float32(8.0), np.float32(0))
    s = ctx.compress(dev(x), atol).cpu().numpy().tobytes()
    assert s == ocodec.compress(x, atol)
    x.flat[17] = -8.0
    with pytest.raises(F.FwiError) as e:
        ctx.compress(dev(x), atol)
    assert e.value.code == F.FWI_ERANGE
    # a compressed schedule whose wavefield exceeds the range: the source
    # node alone carries b q with b = dt^2/m
    shot = synth.tiny_shot(2, n=20, so=4, nbl=4, nt=30)
    m0, _, q = inputs(shot)
    dobs = torch.zeros((shot.nt, len(shot.rec)), device="cuda:0")
    with pytest.raises(F.FwiError) as e:
        ctx.gradient(shot, dev(m0), dev(q * 1e3), dobs, nslots=3, compress=True, atol=2.0 ** -60)
    assert e.value.code == F.FWI_ERANGE


def test_codec_error_paths(ctx):
    x = dev(synth.wavefield_like((20, 20, 20), seed=4))
    s = ctx.compress(x, 1e-4)
    with pytest.raises(F.FwiError) as e:
        ctx.decompress(s[:-8], (20, 20, 20))
    assert e.value.code == F.FWI_ECORRUPT
    bad = s.clone()
    bad[0] = 0
    with pytest.raises(F.FwiError) as e:
        ctx.decompress(bad, (20, 20, 20))
    assert e.value.code == F.FWI_ECORRUPT
    with pytest.raises(F.FwiError) as e:
        ctx.decompress(s, (20, 20, 21))
    assert e.value.code == F.FWI_ECORRUPT
    y = x.clone()
    y[3, 4, 5] = float("nan")
    with pytest.raises(F.FwiError) as e:
        ctx.compress(y, 1e-4)
    assert e.value.code == F.FWI_ENONFINITE
    import ctypes
    out = torch.empty(100, dtype=torch.uint8, device=DEV)
    nb = ctypes.c_size_t()
    rc = F.lib().ckpt_compress(ctx.h, ctypes.c_void_p(x.data_ptr()), 3, F._dims3((20, 20, 20)),
                               1e-4, ctypes.c_void_p(out.data_ptr()), 100, ctypes.byref(nb),
                               F._stream())
    assert rc == F.FWI_ECAPACITY


def test_gradient_error_paths(ctx):
    shot = synth.tiny_shot(2, n=20, so=4, nbl=4, nt=20)
    m0, mt, q = inputs(shot)
    dobs = ctx.forward(shot, dev(mt), dev(q))
    import copy
    bad = copy.copy(shot)
    bad.dt = shot.dt * 2.0
    with pytest.raises(F.FwiError) as e:
        ctx.gradient(bad, dev(m0), dev(q), dobs)
    assert e.value.code == F.FWI_EUNSTABLE
    bad = copy.copy(shot)
    bad.rec = np.array([[0, 2], [20, 2]], np.int32)
    with pytest.raises(F.FwiError) as e:
        ctx.forward(bad, dev(m0), dev(q))
    assert e.value.code == F.FWI_EINVAL
    small = F.Context(0, pool_bytes=1 << 12)
    with pytest.raises(F.FwiError) as e:
        small.gradient(shot, dev(m0), dev(q), dobs, nslots=3)
    assert e.value.code == F.FWI_ECAPACITY
    with pytest.raises(F.FwiError) as e:
        small.gradient(shot, dev(m0), dev(q), dobs, nslots=3, compress=True, atol=1e-6, pool_bytes=256)
    assert e.value.code == F.FWI_ECAPACITY
    small.close()


@pytest.mark.gpu
@pytest.mark.parametrize("width", [4, 8, 16])
@pytest.mark.parametrize("ns,nd", [(1, 1), (3, 1), (5, 2)])
@pytest.mark.parametrize("grid", [37, 0])
def test_bandwidth_probe_sums_sources(width, ns, nd, grid):
    # the probe is the kernel of known traffic behind the counter
    # calibration: every destination must hold the sum of the sources
    import torch
    n = 4096 * 7 + 12          # ragged against the grid stride
    g = torch.Generator().manual_seed(4)
    srcs = [torch.randn(n, generator=g).to("cuda:0") for _ in range(ns)]
    dsts = [torch.zeros(n, device="cuda:0") for _ in range(nd)]
    F.fwi_bandwidth_probe(srcs, dsts, width, grid)
    ref = sum(s.double() for s in srcs)
    for d in dsts:
        assert torch.allclose(d.double(), ref, rtol=0, atol=1e-5)
