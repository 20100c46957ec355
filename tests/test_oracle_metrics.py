"""Error metrics of the paper (Sec. 3 "Error metrics") on hand-computed cases."""
import math

import numpy as np

from oracle import metrics


def test_psnr_known():
    F = np.array([0.0, 1.0, 2.0, 4.0])           # R = 4
    G = F + np.array([0.1, -0.1, 0.1, -0.1])     # MSE = 0.01
    assert math.isclose(metrics.psnr(F, G), 10 * math.log10(16 / 0.01), rel_tol=1e-12)
    assert metrics.psnr(F, F) == math.inf


def test_angle_known_and_tiny():
    assert math.isclose(metrics.angle([1.0, 0.0], [1.0, 1.0]), math.pi / 4, rel_tol=1e-14)
    a = np.array([1.0, 0.0])
    eps = 1e-9
    b = np.array([math.cos(eps), math.sin(eps)])
    assert math.isclose(metrics.angle(a, b), eps, rel_tol=1e-6)


def test_norms_known():
    F = np.array([3.0, 0.0, -1.0])
    G = np.array([0.0, 4.0, -1.0])
    assert metrics.l2(F, G) == 5.0
    assert metrics.linf(F, G) == 4.0
    assert math.isclose(metrics.rel_l2(F, G), 5.0 / math.sqrt(17.0))
