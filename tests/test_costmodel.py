"""Cost model of the checkpointed gradient (paper_2009_12623_amd.costmodel):
schedule counts taken from the library's planner, pinned to the closed form
of binomial checkpointing (Griewank-Walther forward-step count, checked by
brute force in the oracle tests) and to the store-all special case, where
every state but the initial zero one is stored once and nothing is
recomputed."""
import pytest

from oracle import revolve

F = pytest.importorskip("paper_2009_12623_amd.fwigrad")
from paper_2009_12623_amd import costmodel as C  # noqa: E402


@pytest.mark.parametrize("nt,s", [(10, 3), (40, 5), (100, 7), (2000, 40), (2000, 400)])
def test_forward_count_is_binomial_closed_form(nt, s):
    c = C.schedule_counts(F.fwi_revolve_plan, nt, s)
    assert c.forward == revolve.T_closed(nt, s)


@pytest.mark.parametrize("nt", [2, 10, 2000])
def test_store_all_counts(nt):
    c = C.schedule_counts(F.fwi_revolve_plan, nt, nt)
    # u^0 = 0 is never stored; u^1..u^{nt-1} are stored once, restored once
    assert (c.forward, c.encodes, c.restores_uk, c.restores_both, c.peak_fields) == \
        (nt, nt - 1, nt - 1, 0, nt - 1)


@pytest.mark.parametrize("nt,s", [(10, 3), (7, 1), (60, 4), (500, 20)])
def test_counts_are_consistent_with_the_action_list(nt, s):
    acts, _ = F.fwi_revolve_plan(nt, s)
    c = C.schedule_counts(F.fwi_revolve_plan, nt, s)
    takes = sum(a[0] == "takeshot" for a in acts)
    restores = sum(a[0] == "restore" and a[1] >= 0 for a in acts)
    assert c.restores_uk + c.restores_both == restores
    # a checkpoint restored before forward propagation also keeps u^{k-1}
    assert takes <= c.encodes <= 2 * takes
    assert c.encodes - takes == sum(1 for i, a in enumerate(acts) if a[0] == "takeshot"
                                    and _restarted(acts, i))
    assert c.peak_fields <= 2 * s
    assert sum(a[0] == "reverse" for a in acts) == nt


def _restarted(acts, i):
    slot = acts[i][1]
    for j in range(i + 1, len(acts)):
        if acts[j][0] == "free" and acts[j][1] == slot:
            return False
        if acts[j][0] == "restore" and acts[j][1] == slot and acts[j + 1][0] == "advance":
            return True
    return False


def test_prediction_for_store_all_is_the_plain_sum():
    u = C.UnitCosts(t_fwd=1.0, t_adj=2.0, t_enc=0.5, t_dec=0.25, field_bytes=100.0)
    c = C.schedule_counts(F.fwi_revolve_plan, 50, 50)
    assert C.predict_ms(c, u, 50) == pytest.approx(50 * 1.0 + 50 * 2.0 + 49 * 0.5 + 49 * 0.25)


def test_choose_slots_respects_the_budget():
    nt = 400
    u = C.UnitCosts(t_fwd=1.0, t_adj=2.0, t_enc=0.5, t_dec=0.5, field_bytes=1000.0)
    best, table = C.choose_slots(F.fwi_revolve_plan, nt, u, budget_bytes=1e12)
    assert best[0] == nt  # storage free: store everything, recompute nothing
    budget = 130 * 1000.0 * 1.3
    best, table = C.choose_slots(F.fwi_revolve_plan, nt, u, budget_bytes=budget)
    c = C.schedule_counts(F.fwi_revolve_plan, nt, best[0])
    assert c.peak_fields * 1000.0 * 1.3 <= budget
    assert all(t >= best[1] / 1e3 - 1e-9 for _, t in table)
    # a slot count with more storage than the budget is never in the table
    for s, _ in table:
        assert C.schedule_counts(F.fwi_revolve_plan, nt, s).peak_fields * 1300.0 <= budget
    assert C.choose_slots(F.fwi_revolve_plan, nt, u, budget_bytes=1.0)[0] is None


def test_unit_costs_from_stats():
    st = dict(ms_forward=10.0, n_forward=5, ms_adjoint=8.0, n_adjoint=4, ms_encode=3.0,
              n_encode=3, ms_decode=0.0, n_decode=0, ckpt_bytes=300)
    u = C.UnitCosts.from_stats(st)
    assert (u.t_fwd, u.t_adj, u.t_enc, u.t_dec, u.field_bytes) == (2.0, 2.0, 1.0, 0.0, 100.0)


def test_choose_config_trades_tolerance_against_slots():
    nt = 400
    plan = F.fwi_revolve_plan
    tight = C.UnitCosts(t_fwd=1.0, t_adj=2.0, t_enc=0.5, t_dec=0.5, field_bytes=4000.0)
    loose = C.UnitCosts(t_fwd=1.0, t_adj=2.0, t_enc=0.5, t_dec=0.5, field_bytes=1000.0)
    budget = 130 * 1000.0 * 1.3
    atol, s, ms = C.choose_config(plan, nt, {1e-6: tight, 1e-3: loose}, budget)
    # the looser tolerance stores four times more fields in the same budget
    assert atol == 1e-3
    assert ms == pytest.approx(C.predict_ms(C.schedule_counts(plan, nt, s), loose, nt))
    best_tight, _ = C.choose_slots(plan, nt, tight, budget)
    assert best_tight is None or best_tight[1] >= ms
    assert C.choose_config(plan, nt, {1e-6: tight}, 1.0) is None


@pytest.mark.parametrize("nt,s", [(50, 50), (200, 12), (2000, 40)])
def test_overlap_share_is_recovered_from_a_measured_call(nt, s):
    # a call that took the stencil time, both-level restores in full and
    # 40 % of the overlappable codec time gives kappa = 0.4 back; with that
    # kappa the prediction reproduces the call
    u = C.UnitCosts(t_fwd=1.3, t_adj=2.2, t_enc=0.8, t_dec=1.1, field_bytes=1e6)
    c = C.schedule_counts(F.fwi_revolve_plan, nt, s)
    stencil = c.forward * 1.3 + nt * 2.2 + 2 * c.restores_both * 1.1
    hidden = c.encodes * 0.8 + c.restores_uk * 1.1
    k = C.overlap_kappa(c, u, nt, stencil + 0.4 * hidden)
    assert k == pytest.approx(0.4)
    u.kappa = k
    assert C.predict_ms(c, u, nt) == pytest.approx(stencil + 0.4 * hidden)
    # clipped to [0, 1]
    assert C.overlap_kappa(c, u, nt, stencil - 5.0) == 0.0
    assert C.overlap_kappa(c, u, nt, stencil + 3 * hidden) == 1.0


def test_full_overlap_leaves_stencil_and_both_level_restores():
    # kappa = 0: encodes and u^k restores cost nothing; restores of both
    # levels precede forward steps that read them and stay
    u = C.UnitCosts(t_fwd=1.0, t_adj=2.0, t_enc=0.5, t_dec=0.25, field_bytes=100.0, kappa=0.0)
    c = C.schedule_counts(F.fwi_revolve_plan, 60, 4)
    assert c.restores_both > 0
    assert C.predict_ms(c, u, 60) == pytest.approx(c.forward + 120.0 + 2 * c.restores_both * 0.25)


def test_unit_costs_take_stencil_times_from_a_codec_free_call():
    st = dict(ms_forward=300.0, n_forward=200, ms_adjoint=500.0, n_adjoint=200, ms_encode=80.0,
              n_encode=100, ms_decode=90.0, n_decode=90, ckpt_bytes=5e8)
    clean = dict(ms_forward=240.0, n_forward=200, ms_adjoint=400.0, n_adjoint=200)
    u = C.UnitCosts.from_stats(st, clean, kappa=0.3)
    assert (u.t_fwd, u.t_adj, u.t_enc, u.t_dec, u.field_bytes, u.kappa) == (1.2, 2.0, 0.8, 1.0, 5e6, 0.3)
