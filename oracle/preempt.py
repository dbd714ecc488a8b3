"""Preemption threshold of Sec. 3 (and the appendix on the implementation):
which rollout length each worker ends with, computed in closed form from the
workers' per-step durations.

TEST INFRASTRUCTURE ONLY (see the package header).

Rule, as read from Sec. 3: a worker that completes all T steps is counted as
finished in a shared counter; after every step, a worker that has collected
at least T/4 steps stops if at least p% of the *other* workers have finished
(the count reaches ceil(p (W - 1))).  So with F_w the time worker w would
complete its T-th step and tau the need-th smallest F_w, every worker with
F_w <= tau collects T steps and every other one stops at the first step s with
s >= T/4 and c_w(s) >= tau (c_w(s): completion time of its s-th step).
Parity: pinned by hand-worked cases, p = 100% (no preemption), a minimum of
T (no preemption), equal speeds, and a brute-force step-by-step replay.
"""
from __future__ import annotations

import math

import numpy as np


def need_count(world: int, frac: float) -> int:
    """Finished workers that trigger preemption: p% of the other workers."""
    return int(math.ceil(frac * (world - 1) - 1e-12))


def min_steps(T: int, min_frac: float = 0.25) -> int:
    return max(1, int(math.ceil(min_frac * T - 1e-12)))


def lengths(durations, frac: float = 0.6, min_frac: float = 0.25):
    """durations [W][T] (seconds per step) -> rollout length per worker [W]."""
    d = np.asarray(durations, np.float64)
    W, T = d.shape
    c = np.cumsum(d, axis=1)                 # c[w, s-1] = completion time of step s
    F = c[:, -1]
    need = need_count(W, frac)
    if need <= 0:
        tau = 0.0
    elif need > W - 1:
        return np.full(W, T, np.int64)       # never reached by the other workers alone
    else:
        tau = np.sort(F)[need - 1]
    smin = min_steps(T, min_frac)
    out = np.full(W, T, np.int64)
    for w in range(W):
        if F[w] <= tau:
            continue
        s = int(np.searchsorted(c[w], tau, side="left")) + 1   # first s with c(s) >= tau
        out[w] = min(T, max(smin, s))
    return out


def replay(durations, frac: float = 0.6, min_frac: float = 0.25):
    """Brute force: advance every worker step by step in completion-time order,
    updating the finished count as events happen."""
    d = np.asarray(durations, np.float64)
    W, T = d.shape
    need = need_count(W, frac)
    smin = min_steps(T, min_frac)
    steps = np.zeros(W, np.int64)
    t = np.zeros(W)
    active = set(range(W))
    finished = 0
    while active:
        w = min(active, key=lambda k: t[k] + d[k, steps[k]])
        t[w] += d[w, steps[w]]
        steps[w] += 1
        if steps[w] == T:
            finished += 1
            active.discard(w)
        elif steps[w] >= smin and finished >= need:
            active.discard(w)
    return steps
