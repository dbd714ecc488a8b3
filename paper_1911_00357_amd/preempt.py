"""Preemption threshold of Sec. 3: the host-side control plane that ends a
straggler's rollout early.

Every worker holds a `PreemptionMonitor` over one shared key-value store (any
object with `add(key, amount) -> int`, e.g. torch.distributed.TCPStore, as in
the paper's appendix on the implementation).  A worker that completes all T
steps of its rollout adds itself to the iteration's finished count; after
each step, a worker that has collected at least T/4 steps stops once the count
has reached p% of the other workers (p = 60% in the paper).  The resulting
per-worker lengths T_n are what the packed learner consumes, each worker's
contribution weighted 1/(|B| T_n).  Host-only: no device work.
"""
from __future__ import annotations

import math
import time


class PreemptionMonitor:
    def __init__(self, store, world_size: int, T: int, frac: float = 0.6, min_frac: float = 0.25,
                 prefix: str = "ddppo/finished"):
        if world_size < 1 or T < 1 or not 0.0 <= frac <= 1.0 or not 0.0 < min_frac <= 1.0:
            raise ValueError("bad preemption parameters")
        self.store, self.W, self.T = store, world_size, T
        # p% of the *other* workers; a threshold above W-1 can never be reached
        self.need = int(math.ceil(frac * (world_size - 1) - 1e-12))
        self.min_steps = max(1, int(math.ceil(min_frac * T - 1e-12)))
        self.prefix = prefix
        self.key = None
        self.steps = 0

    def begin(self, iteration: int):
        """Start collecting the rollout of `iteration` (keys are per iteration,
        so no reset of the store is needed between iterations)."""
        self.key = f"{self.prefix}/{iteration}"
        self.steps = 0

    def finished_count(self) -> int:
        return int(self.store.add(self.key, 0))

    def after_step(self) -> bool:
        """Call after each collected step; True when this worker's rollout ends
        here (complete, or preempted)."""
        if self.key is None:
            raise RuntimeError("begin() first")
        self.steps += 1
        if self.steps >= self.T:
            self.store.add(self.key, 1)
            return True
        if self.steps >= self.min_steps and self.need <= self.W - 1 and self.finished_count() >= self.need:
            return True
        return False


def collect(monitor: PreemptionMonitor, iteration: int, step_fn) -> int:
    """Run step_fn(t) for t = 0, 1, ... until the monitor ends the rollout;
    returns the rollout length."""
    monitor.begin(iteration)
    t = 0
    while True:
        step_fn(t)
        t += 1
        if monitor.after_step():
            return t


def check_overhead_us(store, n: int = 200) -> float:
    """Mean wall time of one finished-count query on `store` (microseconds)."""
    m = PreemptionMonitor(store, 2, 10 ** 9)
    m.begin(-1)
    t0 = time.perf_counter()
    for _ in range(n):
        m.finished_count()
    return (time.perf_counter() - t0) / n * 1e6
