"""Preemption threshold (Sec. 3): the oracle's closed form against hand-worked
cases and a brute-force replay; the library's store-driven monitor against
the oracle, in simulated time with an in-process store and in real time with
worker processes over a torch.distributed.TCPStore on 127.0.0.1."""
import heapq
import multiprocessing as mp
import socket
import time

import numpy as np
import pytest

from oracle import preempt as O
from paper_1911_00357_amd.preempt import PreemptionMonitor, check_overhead_us


def test_hand_worked_straggler():
    # 5 workers, T = 8: four take 10 ms per step, one 100 ms.  p = 60% of the 4
    # others -> 3 finished needed; they finish at 80 ms; the straggler has 1 step
    # by then, and the floor T/4 = 2 keeps it to 2 steps.
    d = np.full((5, 8), 0.010)
    d[4] = 0.100
    assert list(O.lengths(d)) == [8, 8, 8, 8, 2]


def test_hand_worked_threshold_order():
    # W = 6, T = 12, workers finish at 12, 24, 36, ... ms (1..6 ms per step);
    # need = ceil(0.6 * 5) = 3 -> tau = 36 ms (third finisher).  Worker 3 (4 ms
    # steps) reaches 36 ms at step 9, worker 4 at step ceil(36/5) = 8, worker 5
    # at step 6; all above the floor 3.
    d = np.array([[0.001 * (w + 1)] * 12 for w in range(6)])
    assert list(O.lengths(d)) == [12, 12, 12, 9, 8, 6]


def test_no_preemption_cases():
    g = np.random.default_rng(0)
    d = g.lognormal(0, 1, (7, 20))
    # p = 100% of the others is met only once all six others are done: only the
    # slowest worker can be preempted, and not below T/4 steps
    L = O.lengths(d, frac=1.0)
    slow = int(np.argmax(d.sum(1)))
    assert np.all(np.delete(L, slow) == 20) and 5 <= L[slow] <= 20
    # a floor of T disables preemption
    assert np.all(O.lengths(d, min_frac=1.0) == 20)
    # equal speeds: everyone finishes together, nobody is preempted
    assert np.all(O.lengths(np.full((8, 16), 0.01)) == 16)


@pytest.mark.parametrize("seed", range(6))
def test_closed_form_equals_replay(seed):
    g = np.random.default_rng(seed)
    W, T = int(g.integers(2, 12)), int(g.integers(4, 40))
    d = g.lognormal(0, 1.0, (W, T)) * g.lognormal(0, 1.0, (W, 1))
    for frac in (0.0, 0.3, 0.6, 0.8, 1.0):
        assert np.array_equal(O.lengths(d, frac), O.replay(d, frac)), (W, T, frac)


class DictStore:
    def __init__(self):
        self.v = {}

    def add(self, key, amount):
        self.v[key] = self.v.get(key, 0) + amount
        return self.v[key]


def simulate(d, frac):
    """Drive one monitor per worker in simulated time: each worker's next step
    completion is an event; the store is shared."""
    W, T = d.shape
    store = DictStore()
    mons = [PreemptionMonitor(store, W, T, frac) for _ in range(W)]
    for m in mons:
        m.begin(7)
    ev = [(d[w, 0], w) for w in range(W)]
    heapq.heapify(ev)
    out = np.zeros(W, np.int64)
    while ev:
        t, w = heapq.heappop(ev)
        if mons[w].after_step():
            out[w] = mons[w].steps
        else:
            heapq.heappush(ev, (t + d[w, mons[w].steps], w))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_monitor_matches_oracle_simulated_time(seed):
    g = np.random.default_rng(100 + seed)
    W, T = int(g.integers(2, 16)), int(g.integers(4, 64))
    d = g.lognormal(0, 1.0, (W, T)) * g.lognormal(0, 1.5, (W, 1))
    for frac in (0.0, 0.6, 1.0):
        assert np.array_equal(simulate(d, frac), O.lengths(d, frac))


def _free_port():
    s = socket.socket()
    s.bind(("127.0.0.1", 0))
    p = s.getsockname()[1]
    s.close()
    return p


class _TimedStore:
    """Store proxy that records (start, end, amount, result) of every add."""

    def __init__(self, store):
        self.store, self.log = store, []

    def add(self, key, n):
        t0 = time.monotonic()
        r = self.store.add(key, n)
        self.log.append((t0, time.monotonic(), n, int(r)))
        return r


def _worker(rank, world, port, step_s, T, q):
    from torch.distributed import TCPStore
    from paper_1911_00357_amd.preempt import collect
    store = TCPStore("127.0.0.1", port, world, rank == 0, timeout=__import__("datetime").timedelta(seconds=30))
    timed = _TimedStore(store)
    mon = PreemptionMonitor(timed, world, T)
    store.add("ready", 1)
    while store.add("ready", 0) < world:
        time.sleep(0.001)
    t_start = time.monotonic()
    done = []

    def step(t):
        time.sleep(step_s)
        done.append(time.monotonic())

    n = collect(mon, 0, step)
    q.put((rank, n, t_start, done, timed.log))
    store.add("exit", 1)
    if rank == 0:   # the store's host stays until every client is done
        while store.add("exit", 0) < world:
            time.sleep(0.001)


def test_monitor_over_tcpstore_processes():
    """4 worker processes, T = 24: three take 5 ms per step, one 12 ms.  Two
    finished workers (p = 60% of 3) end the straggler's rollout, after about
    10 of its steps.  Checked on what the processes recorded, so scheduling
    noise cannot fail it (under load a nominally fast worker may be the one
    preempted, and is checked the same way):
      - the store is linearisable: a preempted worker's last query ended after
        the second finisher's add began, and its previous query (if above the
        T/4 floor) began before that add ended;
      - the oracle's closed form on the measured step times (from a common
        start) gives every worker's length within one step (a query and an
        add race within a step)."""
    world, T = 4, 24
    steps = [0.005, 0.005, 0.005, 0.012]
    port = _free_port()
    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    ps = [ctx.Process(target=_worker, args=(r, world, port, steps[r], T, q)) for r in range(world)]
    for p in ps:
        p.start()
    rec = {r: (n, t0, done, log) for r, n, t0, done, log in (q.get(timeout=60) for _ in range(world))}
    for p in ps:
        p.join(timeout=60)
    lens = [rec[r][0] for r in range(world)]
    assert lens[3] < T and sum(n == T for n in lens) >= 2, lens
    floor = int(np.ceil(0.25 * T))
    # the second add of 1 to the finished count (its result is 2)
    adds = sorted((a for r in range(world) for a in rec[r][3] if a[2] == 1), key=lambda a: a[3])
    a_begin, a_end = adds[1][0], adds[1][1]
    for r in range(world):
        n, _, done, log = rec[r]
        assert len(done) == n
        queries = [a for a in log if a[2] == 0]       # one per step from the T/4 floor on
        if n == T:
            assert len(queries) == T - floor and all(a[3] < 2 for a in queries)
            continue
        assert len(queries) == n - floor + 1
        assert queries[-1][1] > a_begin and queries[-1][3] >= 2
        if len(queries) > 1:
            assert queries[-2][0] < a_end and queries[-2][3] < 2
    # the closed form on the measured durations from a common start
    t0 = min(rec[r][1] for r in range(world))
    d = np.zeros((world, T))
    for r in range(world):
        c = np.asarray(rec[r][2]) - t0
        d[r, :len(c)] = np.diff(np.concatenate([[0.0], c]))
        d[r, len(c):] = d[r, :len(c)].mean()          # steps a preempted worker did not take
    want = O.lengths(d)
    assert all(abs(n - int(w)) <= 1 for n, w in zip(lens, want)), (lens, want)


def test_store_check_overhead():
    from torch.distributed import TCPStore
    store = TCPStore("127.0.0.1", _free_port(), 1, True)
    us = check_overhead_us(store, 200)
    assert us < 5000
