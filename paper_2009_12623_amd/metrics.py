"""Error metrics of Sec. 3 ("Error metrics") on device tensors, evaluated in
FP64: PSNR = 10 log10(R^2 / MSE) with R the value range of the reference
field and MSE the mean squared difference; the angle between the two fields
seen as vectors (computed as 2 atan2(|a - b|, |a + b|) of the normalised
vectors: the arccos of the cosine, accurate for tiny angles); L2, relative
L2 and L_inf norms of the difference."""
from __future__ import annotations

import math

import torch


def field_errors(ref: torch.Tensor, test: torch.Tensor) -> dict:
    """Metrics of ``test`` against the reference field ``ref``."""
    a = ref.detach().reshape(-1).double()
    b = test.detach().reshape(-1).double()
    e = a - b
    mse = float((e * e).mean())
    rng = float(a.max() - a.min())
    l2 = float(e.norm())
    na, nb = float(a.norm()), float(b.norm())
    if na == 0.0 or nb == 0.0:
        ang = 0.0 if na == nb else math.pi / 2
    else:
        ua, ub = a / na, b / nb
        ang = 2.0 * math.atan2(float((ua - ub).norm()), float((ua + ub).norm()))
    return {
        "psnr_db": math.inf if mse == 0.0 else 10.0 * math.log10(rng * rng / mse) if rng > 0 else -math.inf,
        "angle_rad": ang,
        "l2": l2,
        "rel_l2": (0.0 if l2 == 0.0 else math.inf) if na == 0.0 else l2 / na,
        "linf": float(e.abs().max()),
    }
