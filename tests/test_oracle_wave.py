"""Pins of the FP64 oracle wave solver against what the mathematics fixes.

Each test checks the oracle against something other than its own formulas:
textbook stencil weights and moment conditions, the consistency order of the
Laplacian on an analytic field, the discrete energy of the undamped scheme,
the homogeneous-medium Green's functions (2D and 3D), adjoint dot-product
tests, a Taylor test of the gradient (paper Sec. 4 "Gradient computation",
linearisation figure) and bitwise equality of checkpointed and store-all
gradients (Sec. 1.3: checkpointing alone keeps bitwise equivalence).
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import revolve, solver

# Central second-derivative weights a_0..a_M, from published tables
# (Fornberg 1988, Table 1) -- typed in, not generated.
TEXTBOOK = {
    4: [Fr(-5, 2), Fr(4, 3), Fr(-1, 12)],
    8: [Fr(-205, 72), Fr(8, 5), Fr(-1, 5), Fr(8, 315), Fr(-1, 560)],
    16: [Fr(-1077749, 352800), Fr(16, 9), Fr(-14, 45), Fr(112, 1485),
         Fr(-7, 396), Fr(112, 32175), Fr(-2, 3861), Fr(16, 315315),
         Fr(-1, 411840)],
}


@pytest.mark.parametrize("so", [4, 8, 16])
def test_fd_weights_match_textbook(so):
    a = solver.fd_coeffs(so)
    ref = np.array([float(f) for f in TEXTBOOK[so]])
    np.testing.assert_allclose(a, ref, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("so", [4, 8, 16])
def test_fd_weights_moment_conditions(so):
    # sum_k a_|k| k^(2j) = 2 for j = 1 (second derivative), 0 for j = 0 and
    # for j = 2..M (all higher even moments cancel: order 2M)
    a = TEXTBOOK[so]
    M = so // 2
    for j in range(0, M + 1):
        s = sum((a[abs(k)] * Fr(k) ** (2 * j) for k in range(-M, M + 1)), Fr(0))
        assert s == (2 if j == 1 else 0), (so, j, s)


@pytest.mark.parametrize("so", [4, 8, 16])
def test_laplacian_consistency_order(so):
    # ||Lap_h f - Lap f||_inf on interior points falls like h^SO
    # grid pairs that keep the error above FP64 round-off
    errs, hs = [], []
    for n in {4: (24, 48), 8: (12, 24), 16: (10, 12)}[so]:
        L = 2 * math.pi
        h = L / n
        x = np.arange(n + 2 * so) * h
        X, Z = np.meshgrid(x, x, indexing="ij")
        k1, k2 = 1.0, 1.0
        f = np.sin(k1 * X + 0.3) * np.cos(k2 * Z + 0.7)
        lap_exact = -(k1 ** 2 + k2 ** 2) * f
        lap = solver.laplacian(f, h, so)
        sl = slice(so, -so)
        errs.append(np.max(np.abs(lap[sl, sl] - lap_exact[sl, sl])))
        hs.append(h)
    slope = math.log(errs[0] / errs[1]) / math.log(hs[0] / hs[1])
    assert abs(slope - so) < 0.3, (so, slope, errs)


@pytest.mark.parametrize("ndim,so", [(2, 4), (2, 16), (3, 8)])
def test_discrete_energy_is_conserved(ndim, so):
    # no damping, no source: E = <m (u^k - u^{k-1}), (u^k - u^{k-1})>
    #                            - dt^2 <Lap u^k, u^{k-1}> is constant
    n = 20 if ndim == 2 else 12
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=0, nt=1)
    rng = np.random.default_rng(1)
    v = 1500 + 800 * rng.random(shot.comp_shape)
    p = solver.Problem(shot, synth.slowness2(v))
    assert not p.eta.any()
    u0 = rng.standard_normal(p.shape)
    u1 = u0 + 0.1 * rng.standard_normal(p.shape)

    def energy(uk, ukm1):
        du = uk - ukm1
        return float(np.sum(p.m * du * du) - p.dt ** 2 * np.sum(solver.laplacian(uk, p.h, so) * ukm1))

    e0 = energy(u1, u0)
    prev, cur = u0, u1
    for _ in range(150):
        prev, cur = cur, p.step(cur, prev)
        e = energy(cur, prev)
    assert abs(e - e0) <= 1e-11 * abs(e0), (e, e0)
    assert np.max(np.abs(cur)) > 0.05   # the field did not die


def _green_3d(q, t, r, c, h):
    return h ** 3 * q(t - r / c) / (4 * math.pi * r)


def _green_2d(q, t, r, c, h):
    if c * t <= r:
        return 0.0
    xi_max = math.acosh(c * t / r)
    val, _ = integrate.quad(lambda xi: q(t - (r / c) * math.cosh(xi)), 0.0, xi_max,
                            limit=200)
    return h ** 2 * val / (2 * math.pi)


def _ricker(f0):
    def q(t):
        a = (math.pi * f0 * (t - 1.5 / f0)) ** 2
        return (1 - 2 * a) * math.exp(-a)
    return q


@pytest.mark.parametrize("ndim", [2, 3])
def test_green_function_homogeneous(ndim):
    # homogeneous medium, receiver at distance r: the trace must match the
    # analytic Green's function convolved with the wavelet (a point source of
    # strength q h^d), with the error falling under refinement of h and dt
    c, f0, tmax = 2000.0, 12.0, 0.30
    errs = []
    for refine in (1, 2):
        h = 20.0 / refine
        n = (24 if ndim == 3 else 40) * refine
        nbl = 12 * refine
        off = 8 * refine
        dt = synth.stable_dt(h, c, ndim, 8, 0.5)
        src = (n // 2,) * ndim
        rec = np.array([(src[0] + off,) + src[1:]], np.int32)
        nt = int(tmax / dt)
        shot = synth.Shot(ndim, (n,) * ndim, h, 8, nbl, nt, dt, c, f0, src, rec)
        p = solver.Problem(shot, np.full(shot.comp_shape, 1.0 / c ** 2))
        d = solver.forward(p)[:, 0]
        # the first reflection off the outer edge arrives after
        # (2 (n/2 + nbl) - off) h / c > tmax
        assert (2 * (n // 2 + nbl) - off) * h / c > tmax
        green = _green_3d if ndim == 3 else _green_2d
        ref = np.array([green(_ricker(f0), k * dt, off * h, c, h) for k in range(1, nt + 1)])
        errs.append(np.linalg.norm(d - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.6 * errs[0], errs
    assert errs[1] < 0.03, errs


def _problem(ndim=2, n=20, so=4, nbl=5, nt=60, seed=3):
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=nbl, nt=nt)
    v0, vt = synth.tiny_models(shot.shape, seed=seed)
    m0 = synth.slowness2(synth.extend(v0, nbl))
    mt = synth.slowness2(synth.extend(vt, nbl))
    return solver.Problem(shot, m0), solver.Problem(shot, mt)


@pytest.mark.parametrize("ndim,so", [(2, 4), (2, 16), (3, 8)])
def test_dot_product_F(ndim, so):
    # <F q, y> = <q, F* y>,  F = P_r A^-1 P_s^T  (Eq. 2)
    p, _ = _problem(ndim, n=16 if ndim == 2 else 10, so=so, nt=40)
    rng = np.random.default_rng(5)
    q = rng.standard_normal(p.nt)
    y = rng.standard_normal((p.nt, len(p.rec)))
    Fq = solver.forward(p, q=q)
    _, Fy = solver.adjoint(p, y, sample_src=True)
    a, b = float(np.sum(Fq * y)), float(np.sum(q * Fy))
    assert abs(a - b) <= 1e-12 * abs(a)


@pytest.mark.parametrize("ndim,so", [(2, 4), (2, 8), (3, 8)])
def test_dot_product_J(ndim, so):
    # <J dm, dd> = <dm, J^T dd>, J^T dd = the gradient formula (Eq. 4)
    p, _ = _problem(ndim, n=16 if ndim == 2 else 10, so=so, nt=40)
    rng = np.random.default_rng(6)
    dm = rng.standard_normal(p.shape) * 1e-8
    dd = rng.standard_normal((p.nt, len(p.rec)))
    _, states = solver.forward(p, keep_states=True)
    Jdm = solver.born(p, dm, states)
    JTdd, _ = solver.adjoint(p, dd, states)
    a, b = float(np.sum(Jdm * dd)), float(np.sum(dm * JTdd))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_taylor_second_order():
    # Phi(m + H dm) - Phi(m) - H <g, dm> = O(H^2): the remainder ratio per
    # halving of H approaches 4 (the paper's linearisation test shows
    # ratios 4.04, 3.94, 3.94, 3.82)
    p, pt = _problem(2, n=24, so=8, nt=80, seed=9)
    d_obs = solver.forward(pt)
    phi0, g, _ = solver.gradient(p, d_obs)
    rng = np.random.default_rng(11)
    from scipy import ndimage
    dm = ndimage.gaussian_filter(rng.standard_normal(p.shape), 2.0) * p.m.mean() * 0.05
    lin = float(np.sum(g * dm))
    rem = []
    for H in [2.0 ** -k for k in range(1, 6)]:
        pp = solver.Problem(p.shot, p.m + H * dm)
        rem.append(abs(solver.objective(pp, d_obs) - phi0 - H * lin))
    ratios = [rem[i] / rem[i + 1] for i in range(len(rem) - 1)]
    assert all(3.6 < r < 4.4 for r in ratios[1:]), ratios
    # first-order remainder (without the gradient term) only halves
    first = [abs(solver.objective(solver.Problem(p.shot, p.m + H * dm), d_obs) - phi0)
             for H in (2.0 ** -4, 2.0 ** -5)]
    assert 1.7 < first[0] / first[1] < 2.3


@pytest.mark.parametrize("ndim,nslots", [(2, 0), (2, 1), (2, 4), (2, 100), (3, 3)])
def test_checkpointing_is_bitwise_exact(ndim, nslots):
    p, pt = _problem(ndim, n=16 if ndim == 2 else 10, so=4, nt=50)
    d_obs = solver.forward(pt)
    phi, g, _ = solver.gradient(p, d_obs)
    phi2, g2 = solver.gradient_checkpointed(p, d_obs, nslots)
    assert phi2 == phi
    assert np.array_equal(g, g2)


def test_lossy_checkpoint_gradient_error_shrinks_with_atol():
    # the error enters only through the forward states used in the imaging
    # condition; it must fall as atol falls and vanish relative to FP32 noise
    p, pt = _problem(2, n=24, so=4, nt=80)
    d_obs = solver.forward(pt)
    phi, g, _ = solver.gradient(p, d_obs)
    errs = []
    for atol in (1e-1, 1e-3, 1e-5):
        phi2, g2 = solver.gradient_checkpointed(p, d_obs, 5, atol=atol)
        assert phi2 == phi     # residuals come from the exact first sweep
        errs.append(np.linalg.norm(g2 - g) / np.linalg.norm(g))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4


def test_schedule_drives_gradient_with_expected_step_count():
    p, pt = _problem(2, n=12, so=4, nt=40)
    d_obs = solver.forward(pt)
    st = {}
    solver.gradient_checkpointed(p, d_obs, 3, stats=st)
    assert st["forward_steps"] == revolve.T_bruteforce(40, 3)
