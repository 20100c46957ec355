"""CPU ORACLE (test infrastructure only) -- error metrics of the paper.

Sec. 3 "Error metrics": PSNR with R = max(F) - min(F) and MSE the mean
squared error; the angle between F and G seen as vectors; L2 and L_inf norms
of E = F - G.  The angle is evaluated in FP64 as 2 atan2(|a - b|, |a + b|)
on the normalised vectors, which is the same angle as arccos of the cosine
but stays accurate for tiny angles.
"""
from __future__ import annotations

import math

import numpy as np


def psnr(F, G) -> float:
    F = np.asarray(F, np.float64)
    G = np.asarray(G, np.float64)
    mse = float(np.mean((F - G) ** 2))
    R = float(F.max() - F.min())
    return math.inf if mse == 0 else 10.0 * math.log10(R * R / mse)


def angle(F, G) -> float:
    a = np.asarray(F, np.float64).ravel()
    b = np.asarray(G, np.float64).ravel()
    a = a / np.linalg.norm(a)
    b = b / np.linalg.norm(b)
    return 2.0 * math.atan2(np.linalg.norm(a - b), np.linalg.norm(a + b))


def l2(F, G) -> float:
    return float(np.linalg.norm(np.asarray(F, np.float64) - np.asarray(G, np.float64)))


def linf(F, G) -> float:
    return float(np.max(np.abs(np.asarray(F, np.float64) - np.asarray(G, np.float64))))


def rel_l2(F, G) -> float:
    """||F - G|| / ||G|| (0 when both vanish, inf when only G does)"""
    G = np.asarray(G, np.float64)
    num, den = l2(F, G), float(np.linalg.norm(G))
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / den
