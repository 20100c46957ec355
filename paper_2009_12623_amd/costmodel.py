"""Performance model of the checkpointed gradient and a budget-driven slot
count (the paper's Sec. 1.5 points to choosing checkpoint numbers from a
model of recomputation vs storage; this is that model for this library).

One gradient with s slots on nt steps costs

    T(s) = F(s) t_fwd + nt t_adj + 2 R2(s) t_dec + kappa (E(s) t_enc + R1(s) t_dec)

where F is the schedule's forward steps, E the fields encoded (a checkpoint
keeps the older leapfrog level only where forward propagation restarts from
it), R1 the restores that decode u^k alone and R2 those that decode both
levels.  The library runs encodes beside the following forward steps and a
decode of u^k alone beside the current adjoint step, on a second stream:
only the share kappa of that codec time shows up, as the stencil steps it
overlaps slowing down (they share the memory system).  A restore of both
levels is followed by forward steps that read them, so its decodes stay on
the critical path.  kappa = 1 is a serial run (codec overlap off); it is
measured from a compressed call against the stencil's own step times
(``overlap_kappa``).  Its checkpoints need at most peak(s) fields at once.
Unit costs come from measured calls (fwi_stats); the schedule counts from
the library's own planner (fwi_revolve_plan), so the model follows exactly
the action list the executor runs.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass
class ScheduleCounts:
    forward: int          # forward steps
    encodes: int          # fields encoded (compressed mode)
    restores_uk: int      # restores that decode u^k only (next action reverses)
    restores_both: int    # restores that decode both levels (next action advances)
    peak_fields: int      # largest number of stored fields at one time


def schedule_counts(plan, nt: int, nslots: int) -> ScheduleCounts:
    """Counts of the binomial schedule; ``plan(nt, nslots)`` returns
    (actions, forward steps) like fwigrad.fwi_revolve_plan."""
    acts, nf = plan(nt, nslots)
    both, taken = {}, {}
    for i, a in enumerate(acts):
        if a[0] == "takeshot":
            taken[a[1]] = i
            both[i] = False
        elif a[0] == "restore" and a[1] >= 0 and i + 1 < len(acts) and acts[i + 1][0] == "advance":
            both[taken[a[1]]] = True
    nenc = rr = ra = 0
    live = {}
    fields = high = 0
    for i, a in enumerate(acts):
        if a[0] == "takeshot":
            lv = 2 if both[i] else 1
            live[a[1]] = lv
            fields += lv
            high = max(high, fields)
            nenc += lv
        elif a[0] == "restore" and a[1] >= 0:
            if i + 1 < len(acts) and acts[i + 1][0] == "reverse":
                rr += 1
            else:
                ra += 1
        elif a[0] == "free":
            fields -= live.pop(a[1])
    return ScheduleCounts(nf, nenc, rr, ra, high)


@dataclass
class UnitCosts:
    t_fwd: float          # ms per forward step
    t_adj: float          # ms per adjoint + imaging step
    t_enc: float          # ms per field encoded
    t_dec: float          # ms per field decoded
    field_bytes: float    # mean compressed bytes per field
    kappa: float = 1.0    # share of overlapped codec time on the critical path

    @classmethod
    def from_stats(cls, st: dict, stencil: dict | None = None, kappa: float = 1.0) -> "UnitCosts":
        """from fwi_stats of a compressed call with per-kernel timing on;
        ``stencil`` (fwi_stats of a call without codec work, e.g. the
        uncompressed run) supplies the stencil step times when given"""
        n = lambda k: max(st[k], 1)
        src = stencil if stencil is not None else st
        m = lambda k: max(src[k], 1)
        return cls(src["ms_forward"] / m("n_forward"), src["ms_adjoint"] / m("n_adjoint"),
                   st["ms_encode"] / n("n_encode"), st["ms_decode"] / n("n_decode"),
                   st["ckpt_bytes"] / n("n_encode"), kappa)


def predict_ms(c: ScheduleCounts, u: UnitCosts, nt: int) -> float:
    return (c.forward * u.t_fwd + nt * u.t_adj + 2 * c.restores_both * u.t_dec
            + u.kappa * (c.encodes * u.t_enc + c.restores_uk * u.t_dec))


def overlap_kappa(c: ScheduleCounts, u: UnitCosts, nt: int, measured_ms: float) -> float:
    """kappa that makes predict_ms equal a measured call of schedule ``c``
    (u: clean stencil step times and that call's codec times), clipped to
    [0, 1]; 1 when the call has no overlappable codec work"""
    hidden = c.encodes * u.t_enc + c.restores_uk * u.t_dec
    if hidden <= 0:
        return 1.0
    base = c.forward * u.t_fwd + nt * u.t_adj + 2 * c.restores_both * u.t_dec
    return min(1.0, max(0.0, (measured_ms - base) / hidden))


CANDIDATES = (40, 50, 64, 80, 100, 128, 160, 200, 256, 320, 400, 512, 640, 800, 1000,
              1280, 1600, 2000, 2500, 3000)


def choose_slots(plan, nt: int, units: UnitCosts, budget_bytes: float, margin: float = 1.3,
                 candidates=CANDIDATES):
    """Fastest predicted slot count whose peak checkpoint storage (peak
    fields x mean field bytes x margin) fits the budget.  Returns
    (best (slots, ms) or None, table of (slots, predicted s))."""
    best, table = None, []
    for s in sorted(set(candidates) | {nt}):
        if s > nt:
            continue
        c = schedule_counts(plan, nt, s)
        if c.peak_fields * units.field_bytes * margin > budget_bytes:
            continue
        t = predict_ms(c, units, nt)
        table.append((s, round(t / 1e3, 3)))
        if best is None or t < best[1]:
            best = (s, t)
    return best, table


def choose_config(plan, nt: int, units_by_atol: dict, budget_bytes: float, margin: float = 1.3,
                  candidates=CANDIDATES):
    """(atol, slots, predicted ms) minimising the predicted time over the
    tolerances the caller accepts (``units_by_atol``: atol -> UnitCosts,
    e.g. from a pilot call per atol: the stream size and codec costs depend
    on atol) and the slot counts that fit the budget; None if nothing fits.
    The choice of an acceptable atol is the caller's (the error it causes is
    not modelled)."""
    best = None
    for atol, units in sorted(units_by_atol.items()):
        b, _ = choose_slots(plan, nt, units, budget_bytes, margin, candidates)
        if b is not None and (best is None or b[1] < best[2]):
            best = (atol, b[0], b[1])
    return best
