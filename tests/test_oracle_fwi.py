"""Pins of the oracle's FWI loop (paper Sec. 4 "Convergence"; the step rule
is the reading taken in oracle/fwi.py).  The descent is driven by an
analytic quadratic objective whose iterates follow in closed form, then run
on a tiny 2D survey with the FP64 wave solver for the properties the rule
guarantees (decrease, mask, bounds, size of the first update)."""
import numpy as np
import pytest

import synth
from oracle import fwi as ofwi
from oracle import solver


def _quadratic(m_star, weight=None):
    w = np.ones_like(m_star) if weight is None else weight

    def value(m):
        return 0.5 * float(np.sum(w * (m - m_star) ** 2))

    def value_and_grad(m):
        return value(m), w * (m - m_star)
    return value_and_grad, value


def test_iterates_of_a_quadratic_follow_the_closed_form():
    # f = |m - m*|^2 / 2, e = m0 - m*: every gradient is parallel to e and
    # is divided by the FIRST gradient norm |e|, with the first length
    # a0 = step min|m0| / max|e/|e||, so without backtracking
    # m_k = m* + e (1 - a0/|e|)^k
    rng = np.random.default_rng(3)
    m_star = 1.0 + rng.random((7, 5))
    e = 0.3 * rng.standard_normal((7, 5))
    m0 = m_star + e
    step = 0.05
    vg, v = _quadratic(m_star)
    out = ofwi.descent(m0, vg, v, 4, step, None, None, np.ones_like(m0))
    ne = np.linalg.norm(e)
    a0 = step * np.min(np.abs(m0)) / np.max(np.abs(e / ne))
    r = a0 / ne
    assert 0 < r < 1
    np.testing.assert_allclose(out["m"], m_star + e * (1 - r) ** 4, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(out["lengths"], [a0] * 4, rtol=1e-14)
    want = [0.5 * ne ** 2 * (1 - r) ** (2 * k) for k in range(5)]
    np.testing.assert_allclose(out["objective"], want, rtol=1e-12)


def test_backtracking_halves_until_the_objective_drops():
    # a first length with r = a0/|e| = 5: the trial overshoots (|1 - r| > 1)
    # until r / 2^j < 2, i.e. j = 2 halvings (r = 1.25 is accepted); the
    # accepted length carries over
    m_star = np.zeros(4)
    e = np.array([1.0, -2.0, 2.0, 4.0])
    ne = np.linalg.norm(e)
    m0 = m_star + e
    vg, v = _quadratic(m_star)
    # a0 = step min|m0| / max|e/|e|| = step * 1 / (4/|e|) = 5 |e|  ->  step = 20
    out = ofwi.descent(m0, vg, v, 1, 20.0, None, None, np.ones(4))
    assert out["lengths"][0] == pytest.approx(5 * ne / 4)
    np.testing.assert_allclose(out["m"], e * (1 - 1.25))
    assert [d > 0 for d in out["decreases"]] == [False, False, True]


def test_exhausted_backtracking_takes_the_last_trial():
    m_star = np.zeros(3)
    e = np.array([1.0, 1.0, 1.0])
    vg, v = _quadratic(m_star)
    out = ofwi.descent(m_star + e, vg, v, 1, 1e4, None, None, np.ones(3), backtracks=2)
    a0 = 1e4 * np.sqrt(3.0)
    assert out["lengths"][0] == pytest.approx(a0 / 4)
    np.testing.assert_allclose(out["m"], e - (a0 / 4) * e / np.sqrt(3.0))
    assert len(out["decreases"]) == 3 and max(out["decreases"]) < 0


def test_mask_and_bounds():
    m_star = np.full((4, 4), 1.0)
    e = np.full((4, 4), 0.5)
    e[0] = 3.0
    mask = np.ones((4, 4))
    mask[:, 0] = 0.0
    vg, v = _quadratic(m_star)
    out = ofwi.descent(m_star + e, vg, v, 3, 0.8, 1.2, None, mask)
    assert np.array_equal(out["m"][:, 0], (m_star + e)[:, 0])
    assert np.all(out["m"] >= 1.2)


def test_tiny_survey_descends_inside_mask_and_bounds():
    base = synth.tiny_shot(2, n=30, so=4, nbl=6, nt=120)
    shots = [synth.Shot(2, base.shape, base.h, base.so, base.nbl, base.nt, base.dt, base.vmax,
                        base.f0, (x, 2), base.rec) for x in (8, 22)]
    v0, vt = synth.tiny_models(base.shape, seed=11)
    m0 = synth.slowness2(synth.extend(v0, base.nbl))
    mt = synth.slowness2(synth.extend(vt, base.nbl))
    q = base.wavelet()
    d_obs = [solver.forward(solver.Problem(s, mt, wavelet=q)) for s in shots]
    mask = np.zeros(base.comp_shape)
    mask[6:-6, 6 + 4:-6] = 1.0
    out = ofwi.run_fwi(shots, m0, q, d_obs, 3, 0.05, 1400.0, 2600.0, mask)
    ph = out["objective"]
    assert all(b < a for a, b in zip(ph, ph[1:]))
    assert np.array_equal(out["m"][mask == 0], m0[mask == 0])
    assert np.all(out["m"] <= 1 / 1400.0 ** 2) and np.all(out["m"] >= 1 / 2600.0 ** 2)
