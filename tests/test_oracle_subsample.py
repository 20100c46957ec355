"""Pins of the oracle's time-subsampled gradient (Sec. 4 "Subsampling"):
factor 1 is the full gradient; the mean of the subsampled gradients over
all phases of one factor is the full gradient again (every step imaged
exactly once across the phases, weight 1/factor x factor); a factor larger
than the number of steps images nothing at phase 0; and the objective is the
one of Eq. 3."""
import numpy as np
import pytest

import synth
from oracle import solver


def problem(ndim=2, n=30, so=8, nt=36, seed=2):
    shot = synth.tiny_shot(ndim, n=n, so=so, nbl=5, nt=nt)
    v0, vt = synth.tiny_models(shot.shape, seed=seed)
    p0 = solver.Problem(shot, synth.slowness2(synth.extend(v0, shot.nbl)))
    pt = solver.Problem(shot, synth.slowness2(synth.extend(vt, shot.nbl)))
    return p0, solver.forward(pt)


def test_factor_one_is_the_full_gradient():
    p, d = problem()
    phi, g, _ = solver.gradient(p, d)
    phi1, g1 = solver.gradient_subsampled(p, d, 1)
    assert phi1 == phi
    assert np.array_equal(g1, g)


@pytest.mark.parametrize("factor", [2, 3, 5])
def test_mean_over_phases_is_the_full_gradient(factor):
    p, d = problem(nt=37)
    _, g, _ = solver.gradient(p, d)
    acc = np.zeros_like(g)
    for ph in range(factor):
        _, gf = solver.gradient_subsampled(p, d, factor, ph)
        acc += gf
    acc /= factor
    assert np.linalg.norm(acc - g) <= 1e-12 * np.linalg.norm(g)


def test_subsampled_gradient_differs_and_stays_correlated():
    p, d = problem(nt=60)
    _, g, _ = solver.gradient(p, d)
    _, g4 = solver.gradient_subsampled(p, d, 4)
    cos = float(np.sum(g * g4) / (np.linalg.norm(g) * np.linalg.norm(g4)))
    assert not np.array_equal(g, g4)
    assert 0.5 < cos < 1.0


def test_factor_above_steps_images_nothing():
    p, d = problem(nt=20)
    phi, g = solver.gradient_subsampled(p, d, 21)
    assert not g.any()
    assert phi == pytest.approx(solver.objective(p, d), rel=1e-15)


def test_bad_arguments():
    p, d = problem(nt=10)
    with pytest.raises(ValueError):
        solver.gradient_subsampled(p, d, 0)
    with pytest.raises(ValueError):
        solver.gradient_subsampled(p, d, 3, 3)
