"""CPU ORACLE (test infrastructure only) -- FP64 forward, adjoint, gradient.

Follows the paper's statement of the problem (Sec. 2):
  d_sim = P_r A(m)^-1 P_s^T q_s          (Eq. 2)
  Phi   = 1/2 || d_sim - d_obs ||^2      (Eq. 3, no dt weight)
  grad  = sum_t u[t] v_tt[t] = J^T (d_sim - d_obs)   (Eq. 4)
discretised as in ``wave.c``: row k of the leapfrog system
  D u^k = (2M + Lap) u^{k-1} - B u^{k-2} + P_s^T q^{k-1},  k = 1..N,
receivers d^k = P_r u^k, and the exact discrete adjoint
  D lam^k = (2M + Lap) lam^{k+1} - B lam^{k+2} + P_r^T r^k,  k = N..1,
  g = -(1/dt^2) sum_k u^k (lam^k - 2 lam^{k+1} + lam^{k+2}),
which is Eq. 4 with v = -lam after summation by parts.  Checkpointing
(Sec. 1.3) follows the action list of ``revolve.schedule``; a compressed
checkpoint stores each of (u^k, u^{k-1}) rounded to float32 and compressed
with the same atol (Sec. 3: only the forward wavefield is compressed).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import codec as ocodec
from . import lib, ptr
from . import revolve

_D = ctypes.c_double


def fd_coeffs(so: int) -> np.ndarray:
    a = np.zeros(so // 2 + 1)
    if lib().or_fd_coeffs(so, ptr(a, _D)) != 0:
        raise ValueError("space order must be 4, 8 or 16")
    return a


def _cl(shape):
    return (ctypes.c_long * 3)(*(list(shape) + [1] * (3 - len(shape))))


def laplacian(u: np.ndarray, h: float, so: int) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    lib().or_laplacian(u.ndim, _cl(u.shape), h, so, ptr(u, _D), ptr(out, _D))
    return out


def damping(shape, nbl: int, h: float, vmax: float) -> np.ndarray:
    eta = np.empty(shape, dtype=np.float64)
    lib().or_damping(len(shape), _cl(shape), nbl, h, vmax, ptr(eta, _D))
    return eta


class Problem:
    """One shot on the computational grid (physical + nbl on every side)."""

    def __init__(self, shot, m: np.ndarray, wavelet: np.ndarray | None = None):
        self.shot = shot
        self.m = np.ascontiguousarray(m, dtype=np.float64)
        self.shape = tuple(self.m.shape)
        if self.shape != tuple(shot.comp_shape):
            raise ValueError("model must live on the computational grid")
        self.ndim, self.h, self.so, self.dt = shot.ndim, shot.h, shot.so, shot.dt
        self.nt = shot.nt
        self.np = int(np.prod(self.shape))
        self.eta = damping(self.shape, shot.nbl, shot.h, shot.vmax)
        self.q = shot.wavelet() if wavelet is None else np.asarray(wavelet, np.float64)
        nbl = shot.nbl
        self.src = int(np.ravel_multi_index(tuple(c + nbl for c in shot.src), self.shape))
        rec = np.asarray(shot.rec, dtype=np.int64) + nbl
        self.rec = np.ravel_multi_index(tuple(rec.T), self.shape).astype(np.int64) \
            if len(rec) else np.zeros(0, np.int64)
        self._cl = _cl(self.shape)

    # one leapfrog row; sparse terms added at node indices (repeats add)
    def step(self, u1, u2, idx=None, val=None, dense=None):
        out = np.empty(self.shape)
        nsp = 0 if idx is None else len(idx)
        idx = np.ascontiguousarray(idx if nsp else np.zeros(1), dtype=np.int64)
        val = np.ascontiguousarray(val if nsp else np.zeros(1), dtype=np.float64)
        dptr = ptr(np.ascontiguousarray(dense), _D) if dense is not None else None
        lib().or_step(self.ndim, self._cl, self.h, self.so, self.dt,
                      ptr(self.m, _D), ptr(self.eta, _D), ptr(u1, _D), ptr(u2, _D),
                      ptr(out, _D), dptr, nsp,
                      idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), ptr(val, _D))
        return out

    def image(self, g, u, l0, l1, l2):
        lib().or_image(self.np, self.dt, ptr(u, _D), ptr(l0, _D), ptr(l1, _D),
                       ptr(l2, _D), ptr(g, _D))

    def zeros(self):
        return np.zeros(self.shape)


# ----------------------------------------------------------------- forward
def forward(p: Problem, keep_states: bool = False, q=None):
    """Receiver traces d (nt x nrec), d[k-1] = u^k at the receivers; with
    ``keep_states`` also the list [u^0, u^1, ..., u^N]."""
    q = p.q if q is None else q
    u2, u1 = p.zeros(), p.zeros()
    d = np.zeros((p.nt, len(p.rec)))
    states = [u1.copy()] if keep_states else None
    for k in range(1, p.nt + 1):
        u = p.step(u1, u2, [p.src], [q[k - 1]])
        d[k - 1] = u.ravel()[p.rec]
        if keep_states:
            states.append(u.copy())
        u2, u1 = u1, u
    return (d, states) if keep_states else d


def adjoint(p: Problem, resid: np.ndarray, states=None, sample_src=False):
    """Reverse sweep with receiver sources ``resid`` (nt x nrec).  Returns the
    gradient (if ``states`` from ``forward(keep_states=True)`` are given)
    and/or the adjoint field sampled at the source, s[n] = lam^{n+1}[src]."""
    l1, l2 = p.zeros(), p.zeros()
    g = p.zeros() if states is not None else None
    srcs = np.zeros(p.nt) if sample_src else None
    for k in range(p.nt, 0, -1):
        l0 = p.step(l1, l2, p.rec, resid[k - 1])
        if g is not None:
            p.image(g, states[k], l0, l1, l2)
        if sample_src:
            srcs[k - 1] = l0.ravel()[p.src]
        l2, l1 = l1, l0
    return g, srcs


def gradient(p: Problem, d_obs: np.ndarray):
    """Store-all FWI gradient: returns (phi, g, d_sim)."""
    d, states = forward(p, keep_states=True)
    r = d - d_obs
    phi = 0.5 * float(np.sum(r * r))
    g, _ = adjoint(p, r, states)
    return phi, g, d


def objective(p: Problem, d_obs: np.ndarray) -> float:
    r = forward(p) - d_obs
    return 0.5 * float(np.sum(r * r))


def born(p: Problem, dm: np.ndarray, states=None) -> np.ndarray:
    """J dm: linearised traces.  Row k of the perturbed system has the
    source -(dm/dt^2)(u^k - 2u^{k-1} + u^{k-2})."""
    if states is None:
        _, states = forward(p, keep_states=True)
    dm = np.ascontiguousarray(dm, dtype=np.float64)
    du2, du1 = p.zeros(), p.zeros()
    dd = np.zeros((p.nt, len(p.rec)))
    zero = p.zeros()
    rhs = np.empty(p.shape)
    for k in range(1, p.nt + 1):
        ukm2 = states[k - 2] if k >= 2 else zero
        lib().or_born_rhs(p.np, p.dt, ptr(dm, _D), ptr(states[k], _D),
                          ptr(states[k - 1], _D), ptr(ukm2, _D), ptr(rhs, _D))
        du = p.step(du1, du2, dense=rhs)
        dd[k - 1] = du.ravel()[p.rec]
        du2, du1 = du1, du
    return dd


# --------------------------------------------------------- checkpointing
def gradient_checkpointed(p: Problem, d_obs: np.ndarray, nslots: int,
                          atol: float | None = None, acts=None, resid=None,
                          stats: dict | None = None):
    """FWI gradient following a binomial schedule with ``nslots`` slots.

    atol None: checkpoints are exact FP64 copies (result must equal the
    store-all gradient bit for bit).  Otherwise each level of a checkpoint
    is rounded to float32 and compressed with ``atol``; a restore
    decompresses and promotes to FP64.  ``resid`` given: use it as the
    adjoint source (J^T resid) instead of d_sim - d_obs; phi is then None."""
    if acts is None:
        acts = revolve.schedule(p.nt, nslots)
    work_k = 0
    cur, prev = p.zeros(), p.zeros()
    reached = 0
    d = np.zeros((p.nt, len(p.rec)))
    slots = {}
    l1, l2 = p.zeros(), p.zeros()
    g = p.zeros()
    r = None
    nbytes = []
    for act in acts:
        op = act[0]
        if op == "advance":
            _, a, b = act
            assert work_k == a
            for k in range(a + 1, b + 1):
                u = p.step(cur, prev, [p.src], [p.q[k - 1]])
                prev, cur = cur, u
                if k > reached:
                    d[k - 1] = cur.ravel()[p.rec]
                    reached = k
            work_k = b
        elif op == "takeshot":
            _, slot, k = act
            assert work_k == k
            if atol is None:
                slots[slot] = (k, cur.copy(), prev.copy())
            else:
                s1 = ocodec.compress(cur.astype(np.float32), atol)
                s2 = ocodec.compress(prev.astype(np.float32), atol)
                nbytes.append(len(s1) + len(s2))
                slots[slot] = (k, s1, s2)
        elif op == "restore":
            _, slot, k = act
            if slot < 0:
                assert k == 0
                cur, prev = p.zeros(), p.zeros()
            else:
                sk, a1, a2 = slots[slot]
                assert sk == k
                if atol is None:
                    cur, prev = a1.copy(), a2.copy()
                else:
                    cur = ocodec.decompress(a1, p.shape).astype(np.float64)
                    prev = ocodec.decompress(a2, p.shape).astype(np.float64)
            work_k = k
        elif op == "reverse":
            _, k = act
            assert work_k == k
            if r is None:
                r = (d - d_obs) if resid is None else resid
            l0 = p.step(l1, l2, p.rec, r[k - 1])
            p.image(g, cur, l0, l1, l2)
            l2, l1 = l1, l0
        elif op == "free":
            slots.pop(act[1])
        else:
            raise ValueError(op)
    phi = None if resid is not None else 0.5 * float(np.sum((d - d_obs) ** 2))
    if stats is not None:
        stats["ckpt_bytes"] = nbytes
        stats["forward_steps"] = revolve.forward_steps(acts)
        stats["d_sim"] = d
    return phi, g


# ------------------------------------------------------------- subsampling
def gradient_subsampled(p: Problem, d_obs: np.ndarray, factor: int, phase: int = 0):
    """Time-subsampled imaging condition, the comparison baseline of Sec. 1
    ("Approximate methods") and Sec. 4 ("Subsampling").  The forward and the
    adjoint sweeps keep every step; the sum of Eq. 4 is taken only over the
    steps k (1..N) with k = phase (mod factor), each term weighted by factor
    so that the sum stays an estimate of the full one.  Only those forward
    states need to be kept.  Returns (phi, g)."""
    if factor < 1 or not 0 <= phase < factor:
        raise ValueError("need factor >= 1 and 0 <= phase < factor")
    d, states = forward(p, keep_states=True)
    r = d - d_obs
    phi = 0.5 * float(np.sum(r * r))
    l1, l2 = p.zeros(), p.zeros()
    g = p.zeros()
    for k in range(p.nt, 0, -1):
        l0 = p.step(l1, l2, p.rec, r[k - 1])
        if k % factor == phase:
            term = p.zeros()
            p.image(term, states[k], l0, l1, l2)
            g += factor * term
        l2, l1 = l1, l0
    return phi, g
