"""CPU ORACLE (test infrastructure only) -- binomial checkpoint schedule.

Checkpointing trades recomputation for storage (paper Sec. 1.3
"Checkpointing", Fig. 2; Revolve is cited there).  Our reverse sweep needs the
forward states x_N, x_{N-1}, ..., x_1 in that order, where
x_k = (u^k, u^{k-1}) and one ADVANCE step maps x_k -> x_{k+1}; x_0 = 0 is
free to restore.  With s checkpoint slots the minimal number of forward
steps obeys

    T(n, 0) = n (n + 1) / 2,   T(0, s) = 0,
    T(n, s) = min_{1 <= j <= n} [ j + T(n - j, s - 1) + T(j - 1, s) ]

(advance j steps and store that state; reverse the n - j later states with
one slot fewer; then the j - 1 earlier ones with all slots).  This is the
classic binomial recurrence for n + 1 steps with s + 1 snapshots (one of
them holding the initial state), whose minimum has the closed form
t l - C(c + t, t - 1) with l = n + 1, c = s + 1 and t the smallest integer
with C(c + t, c) >= l.

Action list (tuples):
    ("advance", a, b)     working state x_a -> x_b
    ("takeshot", slot, k) store working x_k in ``slot`` (slots form a stack)
    ("restore", slot, k)  working <- slot (slot -1 is the zero state x_0)
    ("reverse", k)        adjoint row k, needs working x_k
    ("free", slot)        release the top slot
A restore is listed only when the working state differs from the one needed.
The split is the LARGEST j attaining the minimum.
"""
from __future__ import annotations

import functools
import sys
from math import comb


def T_bruteforce(n: int, s: int) -> int:
    """Minimal forward steps by exhaustive recursion (small n only)."""
    @functools.lru_cache(maxsize=None)
    def t(n, s):
        if n == 0:
            return 0
        if s == 0:
            return n * (n + 1) // 2
        return min(j + t(n - j, s - 1) + t(j - 1, s) for j in range(1, n + 1))
    return t(n, s)


@functools.lru_cache(maxsize=None)
def T_closed(n: int, s: int) -> int:
    if n == 0:
        return 0
    if s == 0:
        return n * (n + 1) // 2
    length, c = n + 1, s + 1
    t = 0
    while comb(c + t, c) < length:
        t += 1
    return t * length - comb(c + t, t - 1)


def split(n: int, s: int) -> int:
    best, arg = None, None
    for j in range(1, n + 1):
        v = j + T_closed(n - j, s - 1) + T_closed(j - 1, s)
        if best is None or v <= best:
            best, arg = v, j
    return arg


def schedule(nsteps: int, nslots: int) -> list:
    """Action list that reverses x_N .. x_1 with ``nslots`` slots."""
    if nsteps < 1 or nslots < 0:
        raise ValueError("need nsteps >= 1 and nslots >= 0")
    acts = []
    st = {"work": 0, "depth": 0}

    def ensure(k, slot):
        if st["work"] != k:
            acts.append(("restore", slot, k))
            st["work"] = k

    def advance(a, b):
        acts.append(("advance", a, b))
        st["work"] = b

    def rev(a, b, s, slot_a):
        # reverse x_b .. x_{a+1}; x_a sits in slot_a (or is the zero state)
        while b > a:
            ensure(a, slot_a)
            if s == 0:
                advance(a, b)
                acts.append(("reverse", b))
                b -= 1
                continue
            j = split(b - a, s)
            m = a + j
            advance(a, m)
            if m == b:
                acts.append(("reverse", b))
                b -= 1
                continue
            slot = st["depth"]
            acts.append(("takeshot", slot, m))
            st["depth"] += 1
            rev(m, b, s - 1, slot)
            ensure(m, slot)
            acts.append(("reverse", m))
            acts.append(("free", slot))
            st["depth"] -= 1
            b = m - 1

    sys.setrecursionlimit(max(sys.getrecursionlimit(), 4 * min(nslots, nsteps) + 200))
    rev(0, nsteps, min(nslots, nsteps), -1)
    return acts


def forward_steps(acts) -> int:
    return sum(a[2] - a[1] for a in acts if a[0] == "advance")
