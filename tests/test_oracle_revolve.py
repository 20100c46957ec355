"""Pins of the oracle's checkpoint schedule.

The schedule must realise the minimal number of forward steps of the
binomial recurrence (checked against exhaustive recursion), visit the
reverse steps N..1 exactly once and in order, and respect the slot budget
(paper Sec. 1.3 "Checkpointing", Fig. 2).
"""
import pytest

from oracle import revolve


def test_closed_form_matches_bruteforce():
    for s in range(0, 7):
        for n in range(0, 61):
            assert revolve.T_closed(n, s) == revolve.T_bruteforce(n, s), (n, s)


def simulate(acts, N, s):
    work, slots, rev = 0, [], []
    for a in acts:
        op = a[0]
        if op == "advance":
            assert a[1] == work and a[2] > a[1]
            work = a[2]
        elif op == "takeshot":
            assert a[1] == len(slots) and a[2] == work
            slots.append(work)
            assert len(slots) <= s
        elif op == "restore":
            if a[1] < 0:
                assert a[2] == 0
            else:
                assert slots[a[1]] == a[2]
            work = a[2]
        elif op == "reverse":
            assert a[1] == work
            rev.append(work)
        elif op == "free":
            assert a[1] == len(slots) - 1
            slots.pop()
    assert rev == list(range(N, 0, -1))
    assert not slots


@pytest.mark.parametrize("N", [1, 2, 3, 7, 20, 45])
@pytest.mark.parametrize("s", [0, 1, 2, 3, 5, 50])
def test_schedule_valid_and_optimal(N, s):
    acts = revolve.schedule(N, s)
    simulate(acts, N, s)
    assert revolve.forward_steps(acts) == revolve.T_bruteforce(N, min(s, N))


def test_large_schedule_counts():
    for N, s in [(500, 10), (2000, 40), (1500, 40)]:
        acts = revolve.schedule(N, s)
        simulate(acts, N, s)
        assert revolve.forward_steps(acts) == revolve.T_closed(N, s)
    # store-all: one forward sweep
    acts = revolve.schedule(300, 299)
    assert revolve.forward_steps(acts) == 300
