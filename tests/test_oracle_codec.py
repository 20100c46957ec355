"""Pins of the oracle codec against properties fixed by arithmetic.

The paper uses ZFP's fixed-accuracy mode, whose contract is that every
decoded value lies within atol of the original (appendix L_inf figure: the
error stays below atol at every setting).  Pins here: exact inversion of the
integer lifting, annihilation of constant and linear data by the detail
coefficients, the per-value error bound on adversarial inputs, bit lengths
and words derived by hand for special blocks, lossless decoding of the block
floating-point integers at tiny atol (checked against an independent numpy
computation), monotone compression factor, and rejection of corrupt streams.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import codec

GOLD = os.path.join(os.path.dirname(__file__), "golden", "codec_constant_blocks.json")


def _tables(stream):
    h = codec.header(stream)
    nchunks = h["nchunks"]
    nsuper = (nchunks + 255) // 256
    b = np.frombuffer(stream, np.uint8)
    sup = np.frombuffer(bytes(b[64:64 + 8 * nsuper]), "<u8")
    rel = np.frombuffer(bytes(b[64 + 8 * nsuper:64 + 8 * nsuper + 4 * nchunks]), "<u4")
    tb = (8 * nsuper + 4 * nchunks + 7) // 8 * 8
    payload = np.frombuffer(bytes(b[64 + tb:]), "<u8")
    starts = np.array([int(sup[c // 256]) + int(rel[c]) for c in range(nchunks)])
    return h, starts, payload


# ---------------------------------------------------------------- lifting
def test_lifting_inverts_exactly_random():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        v = rng.integers(-(2 ** 28), 2 ** 28, 4)
        assert np.array_equal(codec.lift_inv(codec.lift_fwd(v)), v)


@pytest.mark.parametrize("ndim", [2, 3])
def test_block_transform_inverts_and_stays_in_range(ndim):
    rng = np.random.default_rng(1)
    lim = 2 ** 24 - 1
    shape = (4,) * ndim
    cases = [rng.integers(-lim, lim + 1, shape) for _ in range(300)]
    sgn = np.indices(shape).sum(0) % 2 * 2 - 1
    cases += [lim * sgn, -lim * sgn, np.full(shape, lim), np.full(shape, -lim),
              np.zeros(shape, int)]
    for blk in cases:
        c = codec.block_fwd(blk)
        # three axes of at most 2 bits growth each: |c| < 2^30, so the
        # 32-digit negabinary code holds every coefficient
        assert np.max(np.abs(c.astype(np.int64))) < 2 ** (24 + 2 * ndim)
        assert np.array_equal(codec.block_inv(c), blk)


def test_lifting_annihilates_constant_and_linear():
    for a, b in [(0, 8), (80, -24), (-1000, 16), (7 * 8, 0)]:
        v = np.array([a + b * i for i in range(4)])
        L, H, h0, h1 = codec.lift_fwd(v)
        assert h0 == 0 and h1 == 0          # linear data: only DC and linear
        assert L == a + b * 3 // 2           # DC is the mean (exact here)
        assert H == 2 * b                    # pair-mean difference
    L, H, h0, h1 = codec.lift_fwd([5, 5, 5, 5])
    assert (L, H, h0, h1) == (5, 0, 0, 0)


def test_block_transform_is_separable_on_trends():
    # a block that is linear along x only has non-zero coefficients only at
    # (x in {0,1}, y = 0, z = 0)
    x = np.arange(4).reshape(4, 1, 1)
    blk = (16 * x + 64) * np.ones((4, 4, 4), int)
    c = codec.block_fwd(blk)
    nz = np.argwhere(c != 0)
    assert {tuple(i) for i in nz} <= {(0, 0, 0), (1, 0, 0)}


# ------------------------------------------------------------ error bound
def _fields():
    rng = np.random.default_rng(2)
    yield "smooth3d", synth.wavefield_like((21, 18, 30), seed=3)
    yield "noise3d", rng.standard_normal((13, 9, 17)).astype(np.float32)
    yield "smooth2d", synth.wavefield_like((45, 38), seed=4)
    spiky = (rng.standard_normal((22, 15, 11)) * 1e-3).astype(np.float32)
    idx = rng.integers(0, spiky.size, 40)
    spiky.ravel()[idx] = rng.choice([-1, 1], 40) * 1e2
    yield "spiky3d", spiky
    mixed = (rng.standard_normal((17, 25)) * 2.0 ** rng.integers(-30, 8, (17, 25))).astype(np.float32)
    yield "mixed2d", mixed


@pytest.mark.parametrize("atol", [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6])
def test_error_bound_holds(atol):
    for name, x in _fields():
        # the bound is guaranteed when max|x| < atol * 2^23 (the codec never
        # needs more precision than a float32 block holds)
        xs = x if np.max(np.abs(x)) < atol * 2 ** 22 else x * (atol * 2 ** 21 / np.max(np.abs(x)))
        xs = xs.astype(np.float32)
        s = codec.compress(xs, atol)
        y = codec.decompress(s, xs.shape)
        err = np.max(np.abs(y.astype(np.float64) - xs.astype(np.float64)))
        assert err <= atol, (name, atol, err)


def test_error_bound_adversarial_blocks():
    # blocks built to maximise transform gain: alternating signs, a single
    # large value next to tiny ones, values just under a power of two
    rng = np.random.default_rng(3)
    for atol in (2.0 ** -3, 2.0 ** -10, 1e-3, 3e-5):
        for _ in range(30):
            sgn = (np.indices((8, 8, 8)).sum(0) % 2 * 2 - 1).astype(np.float64)
            amp = atol * 2 ** rng.uniform(0, 21)
            x = sgn * amp * (1 - 2.0 ** -23) * rng.choice([1.0, 0.999, 0.5, 0.25], (8, 8, 8))
            x = x.astype(np.float32)
            y = codec.decompress(codec.compress(x, atol), x.shape)
            assert np.max(np.abs(y.astype(np.float64) - x)) <= atol


# ------------------------------------------------------------ bit lengths
def test_zero_field_is_one_bit_per_block():
    for shape in [(8, 8), (9, 13, 5), (4, 4, 4)]:
        s = codec.compress(np.zeros(shape, np.float32), 1e-3)
        h = codec.header(s)
        assert h["payload_bits"] == h["nblocks"]
        assert np.all(codec.decompress(s, shape) == 0)


def test_subthreshold_block_is_skipped():
    # all |x| < 2^emax <= atol: one bit, decodes to zero (within atol)
    x = np.full((4, 4, 4), 0.24, np.float32)          # emax = -1 (|x| < 0.5)
    s = codec.compress(x, 0.5)
    assert codec.header(s)["payload_bits"] == 1
    assert np.all(codec.decompress(s, x.shape) == 0)


def test_golden_constant_blocks():
    gold = json.load(open(GOLD))
    for case in gold["cases"]:
        x = np.full(case["shape"], case["value"], np.float32)
        s = codec.compress(x, case["atol"])
        h, starts, payload = _tables(s)
        assert h["magic"] == b"FWZ1"
        assert h["payload_bits"] == case["payload_bits"]
        assert [hex(int(w)) for w in payload] == case["payload_words"]
        assert starts[0] == case["chunk0_offset"]
        assert np.all(starts[1:] == case["other_chunk_offsets"])
        assert np.all(codec.decompress(s, x.shape) == case["value"])


def _negabinary_digits(v):
    # textbook base -2 expansion by repeated division
    d = []
    while v != 0:
        r = v % 2
        d.append(r)
        v = (v - r) // -2
    return d


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("value,atol", [(1.0, 2.0 ** -10), (-3.25, 1e-4), (0.7, 1e-6),
                                        (1e4, 1.0), (5e-3, 1e-4), (-1.5e-2, 2e-3)])
def test_constant_block_length_closed_form(ndim, value, atol):
    # a constant block keeps only its DC coefficient, I = trunc(v 2^(24-emax));
    # with f the top negabinary digit of I, P the lowest plane and S the first
    # coded plane the length is 12 + (S - f) + 2 + 2 (f - P), or
    # 12 + (S - P + 1) if no digit is at or above P
    size, tp, guard = (64, 31, 5) if ndim == 3 else (16, 29, 4)
    x = np.full((4,) * ndim, value, np.float32)
    mant, e = np.frexp(np.float64(x.flat[0]))      # |x| < 2^e
    emax = int(e)
    minexp = math.floor(math.log2(atol))
    s = codec.compress(x, atol)
    bits = codec.header(s)["payload_bits"]
    if emax <= minexp:
        assert bits == 1
        return
    I = int(math.trunc(float(x.flat[0]) * 2.0 ** (24 - emax)))
    digits = _negabinary_digits(I)
    P = max(0, minexp - emax + 24 - guard)
    f = max((i for i, b in enumerate(digits) if b and i >= P), default=-1)
    z = 7 if f < 0 else min(7, tp - f)
    S = tp - z
    expect = 12 + (S - P + 1) if f < 0 else 12 + (S - f) + 2 + 2 * (f - P)
    assert bits == expect
    y = codec.decompress(s, x.shape)
    assert np.max(np.abs(y - x)) <= atol


@pytest.mark.parametrize("shape", [(4, 4), (13, 7), (3, 5, 6), (9, 4, 11)])
def test_tiny_atol_decodes_block_floating_point_exactly(shape):
    # with every plane kept the decoder must return trunc(x 2^(24-emax))
    # 2^(emax-24) with emax the block's exponent -- computed here with numpy.
    # Every plane is kept when the lowest plane minexp - emax + 24 - G is
    # <= 0 for every block while emax stays within the accuracy range
    # (emax <= minexp + 23): |x| in [1/2, 4) at atol 2^-20 (emax 0..2)
    rng = np.random.default_rng(4)
    x = (rng.uniform(0.5, 4.0, shape) * rng.choice([-1.0, 1.0], shape)).astype(np.float32)
    y = codec.decompress(codec.compress(x, 2.0 ** -20), shape)
    nd = len(shape)
    pad = [(0, (-n) % 4) for n in shape]
    xp = np.pad(x.astype(np.float64), pad, mode="edge")
    ref = np.empty_like(xp)
    for bi in np.ndindex(*[n // 4 for n in xp.shape]):
        sl = tuple(slice(4 * b, 4 * b + 4) for b in bi)
        blk = xp[sl]
        e = int(np.max(np.frexp(blk)[1][blk != 0])) if np.any(blk != 0) else 0
        ref[sl] = np.trunc(blk * 2.0 ** (24 - e)) * 2.0 ** (e - 24)
    ref = ref[tuple(slice(0, n) for n in shape)].astype(np.float32)
    assert np.array_equal(y, ref)


def test_compression_factor_monotone_in_atol():
    x = synth.wavefield_like((40, 36, 44), seed=5)
    sizes = [len(codec.compress(x, a)) for a in (1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1)]
    assert all(sizes[i] >= sizes[i + 1] for i in range(len(sizes) - 1)), sizes


def test_bound_is_never_exceeded():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((12, 12, 12)).astype(np.float32) * 1e3
    s = codec.compress(x, 2.0 ** -11)     # every plane of most blocks coded
    assert len(s) <= codec.bound(x.shape)


# --------------------------------------------------------- bad streams
def test_corrupt_streams_rejected():
    x = synth.wavefield_like((10, 9, 8), seed=6)
    s = bytearray(codec.compress(x, 1e-3))
    with pytest.raises(codec.CodecError):
        codec.decompress(bytes(s[:-8]), x.shape)          # truncated payload
    bad = bytearray(s)
    bad[0] = ord("X")
    with pytest.raises(codec.CodecError):
        codec.decompress(bytes(bad), x.shape)             # magic
    with pytest.raises(codec.CodecError):
        codec.decompress(bytes(s), (10, 9, 9))            # wrong dims


def test_nonfinite_and_bad_atol_rejected():
    x = np.zeros((4, 4), np.float32)
    x[1, 2] = np.inf
    with pytest.raises(codec.CodecError):
        codec.compress(x, 1e-3)
    with pytest.raises(codec.CodecError):
        codec.compress(np.zeros((4, 4), np.float32), 0.0)


@pytest.mark.parametrize("shape,log2k", [((5, 6, 7), 0), ((1081, 481), 1), ((200, 200, 200), 2),
                                         ((4100, 4100), 6)])
def test_header_records_chunk_length(shape, log2k):
    """blocks per chunk shrink with the field so that small fields still
    split into at least 16384 chunks; the header records log2 of it and the
    chunk count matches"""
    x = synth.wavefield_like(shape, seed=3) if np.prod(shape) < 3e7 else np.zeros(shape, np.float32)
    h = codec.header(codec.compress(x, 1e-3))
    nblocks = int(np.prod([(n + 3) // 4 for n in shape]))
    k = 1 << log2k
    assert h["log2k"] == log2k
    assert h["nchunks"] == 64 * -(-nblocks // (64 * k))
    kmax = 16 if len(shape) == 3 else 64
    assert k == 1 or -(-nblocks // k) >= 16384               # enough chunks
    assert k == kmax or -(-nblocks // (2 * k)) < 16384        # and no more halving than needed


@pytest.mark.parametrize("ndim", [2, 3])
def test_values_beyond_the_accuracy_range_are_refused(ndim):
    # Sec. 1.4 fixed accuracy: |x - x_hat| <= atol needs every |x| below
    # 2^(floor(log2 atol) + 23); at atol = 2^-20 that limit is 8.  A field
    # just below it keeps the bound (all planes coded, only the 24-bit
    # conversion error remains); one value at the limit is refused.
    atol = 2.0 ** -20
    shape = (9, 6, 7) if ndim == 3 else (13, 10)
    rng = np.random.default_rng(31)
    x = rng.uniform(-1, 1, shape).astype(np.float32)
    x.flat[17] = np.nextafter(np.float32(8.0), np.float32(0))
    y = codec.decompress(codec.compress(x, atol), shape)
    assert np.max(np.abs(y.astype(np.float64) - x)) <= atol
    x.flat[17] = -8.0
    with pytest.raises(codec.CodecError) as e:
        codec.compress(x, atol)
    assert e.value.code == codec.ERANGE
    # a larger atol accepts the same field
    codec.compress(x, 2.0 ** -19)
