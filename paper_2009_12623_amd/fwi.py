"""Gradient-descent FWI on the differentiable batched path (Sec. 4
"Convergence"; gradient scaling as in the experimental setup).

Each iteration evaluates the objective of Eq. (3) summed over shots and its
gradient (Eq. 4) through ``forward_modelling_batch`` (one batched sweep,
checkpoints compressed at ``atol`` or exact) and scales the gradient by the
norm of the first iteration's gradient.  The paper does not state its step
rule; here the first trial step is sized so that its largest update is
``step`` times the smallest squared slowness of the starting model, and a
step that does not lower the objective is halved (up to ``backtracks``
times, each trial a forward-only evaluation; after the last halving the
trial is taken as it is); the accepted length carries over to the next
iteration.  Updates are projected onto the velocity bounds.
``mask`` (same shape as the model, optional) multiplies the gradient, e.g.
to keep the absorbing layer and the acquisition rows fixed.
"""
from __future__ import annotations

import time

import torch

from . import fwigrad as F


def objective_and_gradient(ctx, m, shots, wavelet, d_obs, nslots, compress, atol):
    """(sum over shots of 1/2 ||d_sim - d_obs||^2, its gradient) at m"""
    x = m.detach().clone().requires_grad_(True)
    ds = F.forward_modelling_batch(ctx, x, shots, wavelet, nslots=nslots, compress=compress, atol=atol)
    loss = None
    for d, o in zip(ds, d_obs):
        r = d - o
        term = 0.5 * (r * r).sum()
        loss = term if loss is None else loss + term
    loss.backward()
    return float(loss.detach()), x.grad


def objective(ctx, m, shots, wavelet, d_obs):
    """sum over shots of 1/2 ||d_sim - d_obs||^2 at m (forward sweeps only)"""
    tot = 0.0
    for s, o in zip(shots, d_obs):
        r = (ctx.forward(s, m, wavelet) - o).double()
        tot += 0.5 * float((r * r).sum())
    return tot


def run_fwi(ctx, shots, m0, wavelet, d_obs, iterations=30, nslots=40, compress=True, atol=1e-4,
            step=0.05, vmin=None, vmax=None, mask=None, backtracks=6):
    """Returns a dict with the objective before each iteration and after the
    last (``objective``, iterations + 1 values), the final model ``m``, the
    first gradient norm, the accepted step lengths and the wall time per
    iteration."""
    m = m0.detach().clone()
    lo = None if vmax is None else 1.0 / (vmax * vmax)
    hi = None if vmin is None else 1.0 / (vmin * vmin)

    def project(x):
        return x if lo is None and hi is None else x.clamp(min=lo, max=hi)

    phis, steps, scale, alpha = [], [], None, None
    t0 = time.time()
    phi, g = objective_and_gradient(ctx, m, shots, wavelet, d_obs, nslots, compress, atol)
    for it in range(iterations):
        phis.append(phi)
        if mask is not None:
            g = g * mask
        if scale is None:
            scale = float(g.double().norm())
            if scale == 0.0:
                break
            alpha = step * float(m0.abs().min()) / float((g / scale).abs().max())
        d = g / scale
        for k in range(backtracks + 1):
            trial = project(m - alpha * d)
            phi_t = objective(ctx, trial, shots, wavelet, d_obs)
            if phi_t < phi or k == backtracks:
                break
            alpha *= 0.5
        m = trial
        steps.append(alpha)
        if it + 1 < iterations:
            phi, g = objective_and_gradient(ctx, m, shots, wavelet, d_obs, nslots, compress, atol)
        else:
            phi = phi_t
    torch.cuda.synchronize()
    t_iter = (time.time() - t0) / max(len(phis), 1)
    phis.append(phi)
    return {"objective": phis, "m": m, "grad_norm0": scale, "steps": steps, "s_per_iteration": t_iter}
