"""The package's device-side error metrics agree with the oracle's
(Sec. 3 "Error metrics") on random fields, and with closed forms."""
import math

import numpy as np
import pytest
import torch

from oracle import metrics as om
from paper_2009_12623_amd import metrics as pm


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    F = rng.normal(size=(17, 9, 5))
    G = F + 1e-3 * rng.normal(size=F.shape)
    r = pm.field_errors(torch.from_numpy(F), torch.from_numpy(G))
    assert r["psnr_db"] == pytest.approx(om.psnr(F, G), rel=1e-12)
    assert r["angle_rad"] == pytest.approx(om.angle(F, G), rel=1e-9)
    assert r["l2"] == pytest.approx(om.l2(F, G), rel=1e-12)
    assert r["rel_l2"] == pytest.approx(om.rel_l2(G, F), rel=1e-12)
    assert r["linf"] == pytest.approx(om.linf(F, G), rel=1e-12)


def test_closed_forms():
    F = torch.tensor([0.0, 4.0, 0.0, 0.0])
    G = torch.tensor([0.0, 4.0, 0.0, 0.2])
    r = pm.field_errors(F, G)
    assert r["psnr_db"] == pytest.approx(10 * math.log10(16 / (0.04 / 4)))
    assert r["angle_rad"] == pytest.approx(math.atan2(0.2, 4.0))
    assert r["linf"] == pytest.approx(0.2)
    assert pm.field_errors(F, F)["psnr_db"] == math.inf
    assert pm.field_errors(F, 2 * F)["angle_rad"] == 0.0
