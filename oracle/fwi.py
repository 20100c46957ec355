"""CPU ORACLE (test infrastructure only) -- FP64 gradient-descent FWI loop.

The paper's inversion experiment (Sec. 4 "Convergence"; gradients scaled as
in Sec. 3's setup) runs gradient descent on the squared slowness with the
objective of Eq. (3) summed over shots and the gradient of Eq. (4).  Its step
rule is not stated; the reading followed here (written independently of the
GPU loop):

1. the gradient is multiplied by a mask (zero in the absorbing layer and
   the rows next to the acquisition) and divided by the norm of the first
   iteration's masked gradient, so the first search direction has unit
   norm;
2. the first trial step length is chosen so that the largest entry of the
   first update equals ``step`` times the smallest squared slowness of the
   starting model; later iterations start from the last accepted length;
3. a trial model is the current one moved against the direction and
   clipped to the squared slownesses of the velocity bounds; it is accepted
   when its objective is below the current one, otherwise the length is
   halved and the trial repeated, at most ``backtracks`` times, after which
   the last trial is taken as it is.

``descent`` is that rule for any objective/gradient pair; ``run_fwi`` runs
it with the FP64 wave solver (store-all gradient, summed over shots).
"""
from __future__ import annotations

import numpy as np

from . import solver


def descent(m0, value_and_grad, value, iterations, step, lower, upper, mask, backtracks=6):
    """Projected, scaled gradient descent with halving line search.

    ``value_and_grad(m) -> (phi, g)``; ``value(m) -> phi``; ``lower`` /
    ``upper`` are bounds on m (either may be None); ``mask`` multiplies the
    gradient.  Returns a dict: objective before each iteration and after
    the last, final model, accepted lengths, and for every trial the
    relative decrease (phi - phi_trial) / phi it produced."""
    m = np.array(m0, dtype=np.float64, copy=True)
    m_min = float(np.min(np.abs(m0)))
    history, lengths, decreases = [], [], []
    norm0 = None
    length = None

    def clip(x):
        if lower is not None:
            x = np.maximum(x, lower)
        if upper is not None:
            x = np.minimum(x, upper)
        return x

    phi, g = value_and_grad(m)
    for it in range(iterations):
        history.append(phi)
        gm = g * mask
        if norm0 is None:
            norm0 = float(np.sqrt(np.sum(gm * gm)))
            if norm0 == 0.0:
                break
            length = step * m_min / float(np.max(np.abs(gm / norm0)))
        direction = gm / norm0
        tries = 0
        while True:
            trial = clip(m - length * direction)
            phi_trial = value(trial)
            decreases.append((phi - phi_trial) / phi)
            if phi_trial < phi or tries == backtracks:
                break
            length *= 0.5
            tries += 1
        m = trial
        lengths.append(length)
        if it == iterations - 1:
            phi = phi_trial
        else:
            phi, g = value_and_grad(m)
    history.append(phi)
    return {"objective": history, "m": m, "lengths": lengths, "decreases": decreases,
            "grad_norm0": norm0}


def run_fwi(shots, m0, wavelet, d_obs, iterations, step, vmin, vmax, mask, backtracks=6):
    """The descent on shots sharing one computational grid: the objective is
    the sum of the shots' Eq. (3) values, the gradient the sum of their
    Eq. (4) gradients (exact, store-all), all in FP64."""
    q = np.asarray(wavelet, dtype=np.float64)

    def value_and_grad(m):
        tot, gsum = 0.0, np.zeros_like(m)
        for s, d in zip(shots, d_obs):
            phi, g, _ = solver.gradient(solver.Problem(s, m, wavelet=q), d)
            tot += phi
            gsum += g
        return tot, gsum

    def value(m):
        return sum(solver.objective(solver.Problem(s, m, wavelet=q), d) for s, d in zip(shots, d_obs))

    return descent(m0, value_and_grad, value, iterations, step,
                   None if vmax is None else 1.0 / (vmax * vmax),
                   None if vmin is None else 1.0 / (vmin * vmin), mask, backtracks)
