"""The error and compressibility experiments of Sec. 4 on the GPU path.

Each function runs one experiment through the C ABI (via ``fwigrad``) and
returns plain rows; the error metrics are those of Sec. 3 (``metrics``).
Inputs are device tensors on the computational grid, as for ``fwigrad``.

* ``compressibility_over_time`` -- CF of the forward wavefield as the wave
  spreads ("Evolution of compressibility").
* ``lossy_restart`` -- forward propagation continued from a compressed
  state against the exact continuation ("Forward propagation").
* ``gradient_error_vs_atol`` -- lossy against exact gradient per atol
  ("Gradient computation").
* ``gradient_error_vs_slots`` -- the same per number of checkpoints
  ("Gradient error" against checkpoints).
* ``subsampling_error`` -- the time-subsampled imaging baseline per factor
  ("Subsampling").
* ``stacking_error`` -- the error of the sum over shots of lossy gradients
  as shots are added ("Stacking").
"""
from __future__ import annotations

import torch

from . import fwigrad as F
from .metrics import field_errors


def _round(d: dict, nd=6) -> dict:
    return {k: (float("%.*g" % (nd, v)) if isinstance(v, float) else v) for k, v in d.items()}


def compressibility_over_time(ctx, shot, m, wavelet, atol: float, every: int, stop: int | None = None):
    """Rows (step k, CF of u^k at atol) every ``every`` steps up to ``stop``
    (default nt), advancing one forward sweep with fwi_forward_span."""
    nt = shot.nt if stop is None else int(stop)
    u1, u0 = torch.zeros_like(m), torch.zeros_like(m)
    raw = 4.0 * m.numel()
    rows, k = [], 0
    while k < nt:
        k1 = min(k + every, nt)
        ctx.forward_span(shot, m, wavelet, k, k1, u1, u0)
        k = k1
        nb = ctx.compress(u1, atol).numel()
        rows.append({"step": k, "cf": round(raw / nb, 3), "bytes": nb})
    return rows


def _refused(atol, **kw):
    """row of a tolerance the codec refuses: the field holds values at or
    above atol 2^23, where |x - x_hat| <= atol cannot be guaranteed"""
    return dict({"atol": atol, "refused": "FWI_ERANGE"}, **kw)


def lossy_restart(ctx, shot, m, wavelet, k0: int, atols, k1: int | None = None):
    """Advance to step k0, compress both leapfrog levels at each atol, and
    continue to k1 (default nt) from the decompressed state; rows of the
    errors of u^k1 and of the traces recorded after the restart against the
    exact continuation, with the CF of the restart state."""
    k1 = shot.nt if k1 is None else int(k1)
    u1, u0 = torch.zeros_like(m), torch.zeros_like(m)
    ctx.forward_span(shot, m, wavelet, 0, k0, u1, u0)
    nrec = len(shot.rec)
    d_ex = torch.zeros((shot.nt, nrec), device=m.device)
    e1, e0 = u1.clone(), u0.clone()
    ctx.forward_span(shot, m, wavelet, k0, k1, e1, e0, d_ex)
    rows = []
    for atol in atols:
        try:
            s1, s0 = ctx.compress(u1, atol), ctx.compress(u0, atol)
        except F.FwiError as e:
            if e.code != F.FWI_ERANGE:
                raise
            rows.append(_refused(atol))
            continue
        cf = 2 * 4.0 * m.numel() / (s1.numel() + s0.numel())
        a1, a0 = ctx.decompress(s1, m.shape), ctx.decompress(s0, m.shape)
        start = field_errors(u1, a1)
        d = torch.zeros_like(d_ex)
        ctx.forward_span(shot, m, wavelet, k0, k1, a1, a0, d)
        r = {"atol": atol, "cf": round(cf, 3),
             "restart_psnr_db": round(start["psnr_db"], 3), "restart_linf": start["linf"]}
        for tag, (ref, x) in {"final": (e1, a1), "traces": (d_ex[k0:k1], d[k0:k1])}.items():
            er = field_errors(ref, x)
            r.update({tag + "_psnr_db": round(er["psnr_db"], 3), tag + "_rel_l2": er["rel_l2"],
                      tag + "_linf": er["linf"]})
        rows.append(_round(r))
    return rows


def gradient_error_vs_atol(ctx, shot, m, wavelet, d_obs, atols, nslots: int | None = None):
    """Lossy against exact gradient for each atol (store-all slots unless
    ``nslots``); rows with CF and the metrics of Sec. 3."""
    s = shot.nt if nslots is None else nslots
    phi_ex, g_ex = ctx.gradient(shot, m, wavelet, d_obs, nslots=s)
    g_ex = g_ex.clone()
    rows = []
    for atol in atols:
        try:
            phi, g = ctx.gradient(shot, m, wavelet, d_obs, nslots=s, compress=True, atol=atol)
        except F.FwiError as e:
            if e.code != F.FWI_ERANGE:
                raise
            rows.append(_refused(atol, nslots=s))
            continue
        st = ctx.stats()
        er = field_errors(g_ex, g)
        rows.append(_round({"atol": atol, "nslots": s,
                            "cf": st["ckpt_raw_bytes"] / max(st["ckpt_bytes"], 1),
                            "psnr_db": er["psnr_db"], "angle_rad": er["angle_rad"],
                            "rel_l2": er["rel_l2"], "linf": er["linf"],
                            "phi_rel_err": abs(phi - phi_ex) / phi_ex}))
    return rows


def gradient_error_vs_slots(ctx, shot, m, wavelet, d_obs, slots, atols):
    """PSNR (and the other metrics) of the lossy gradient against the exact
    one for each (atol, number of checkpoints)."""
    _, g_ex = ctx.gradient(shot, m, wavelet, d_obs, nslots=shot.nt)
    g_ex = g_ex.clone()
    rows = []
    for atol in atols:
        for s in slots:
            try:
                _, g = ctx.gradient(shot, m, wavelet, d_obs, nslots=s, compress=True, atol=atol)
            except F.FwiError as e:
                if e.code != F.FWI_ERANGE:
                    raise
                rows.append(_refused(atol, nslots=s))
                continue
            st = ctx.stats()
            er = field_errors(g_ex, g)
            rows.append(_round({"atol": atol, "nslots": s, "forward_steps": st["n_forward"],
                                "psnr_db": er["psnr_db"], "angle_rad": er["angle_rad"],
                                "rel_l2": er["rel_l2"]}))
    return rows


def subsampling_error(ctx, shot, m, wavelet, d_obs, factors):
    """Time-subsampled imaging against the exact gradient per factor; the
    memory reduction (CF) is nt over the number of states kept."""
    _, g_ex = ctx.gradient(shot, m, wavelet, d_obs, nslots=shot.nt)
    g_ex = g_ex.clone()
    rows = []
    for f in factors:
        _, g = ctx.gradient_subsampled(shot, m, wavelet, d_obs, f)
        kept = sum(1 for k in range(1, shot.nt + 1) if k % f == 0)
        er = field_errors(g_ex, g)
        rows.append(_round({"factor": f, "cf": shot.nt / max(kept, 1), "psnr_db": er["psnr_db"],
                            "angle_rad": er["angle_rad"], "rel_l2": er["rel_l2"], "linf": er["linf"]}))
    return rows


def stacking_error(ctx, shots, models, wavelet, d_obs, atol: float, nslots: int, dims=None,
                   origins=None, group: int | None = None, counts=None):
    """Stack (sum over shots, Sec. 4 "Stacking") of the first n lossy
    gradients against the stack of the first n exact ones.  Shots sharing
    one grid stack their whole gradients; crops of one model (``dims``: the
    model's physical shape, ``origins``: each crop's physical origin in it)
    stack their physical parts placed at their origins, as the library's
    fwi_gradient_stack does.  Exact gradients run ``group`` shots per batched
    call (bounds the exact checkpoints' memory); ``counts`` (default
    1..len) lists the n reported."""
    n = len(shots)
    group = n if group is None else group
    g_lo = ctx.gradient_batch(shots, models, wavelet, d_obs, nslots=nslots, compress=True, atol=atol)[1]
    g_ex = []
    for i in range(0, n, group):
        j = min(n, i + group)
        g_ex += [g.clone() for g in ctx.gradient_batch(shots[i:j], models[i:j], wavelet, d_obs[i:j],
                                                       nslots=nslots)[1]]

    def place(acc, g, i):
        if origins is None:
            acc += g.double()
            return
        nb = shots[i].nbl
        phys = g[tuple(slice(nb, -nb) if nb else slice(None) for _ in range(g.dim()))]
        sl = tuple(slice(o, o + w) for o, w in zip(origins[i], phys.shape))
        acc[sl] += phys.double()

    shape = tuple(g_ex[0].shape) if origins is None else tuple(dims)
    se = torch.zeros(shape, dtype=torch.float64, device=g_ex[0].device)
    sl = torch.zeros_like(se)
    want = set(range(1, n + 1) if counts is None else counts)
    rows = []
    for k, (a, b) in enumerate(zip(g_ex, g_lo)):
        place(se, a, k)
        place(sl, b, k)
        if k + 1 in want:
            er = field_errors(se, sl)
            rows.append(_round({"shots": k + 1, "psnr_db": er["psnr_db"], "angle_rad": er["angle_rad"],
                                "rel_l2": er["rel_l2"]}))
    return rows


__all__ = ["compressibility_over_time", "lossy_restart", "gradient_error_vs_atol",
           "gradient_error_vs_slots", "subsampling_error", "stacking_error"]
