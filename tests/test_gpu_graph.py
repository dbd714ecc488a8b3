"""The act loop as one HIP graph that the library captures and owns
(ppo_collect): every launch (with eager library work and synchronisations
between launches) reproduces the eager rollout bitwise, for equal and ragged
rollout lengths, on the caller's stream, whole or one step per call."""
import numpy as np
import pytest
import torch

from synth import rollout as R
from tests.nets import MINI_RESNET
from tests.test_gpu_parity import say

pytestmark = pytest.mark.gpu


def _env(net, T, N, seed, dev):
    g = np.random.default_rng(seed)
    t = lambda a: torch.as_tensor(a).to(dev)
    return {"obs": t(g.random((T + 1, N, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32)),
            "goal": t(g.standard_normal((T + 1, N, 2)).astype(np.float32)),
            "mask": t((g.random((T + 1, N)) > 0.1).astype(np.float32)),
            "u": t(g.random((T + 1, N)).astype(np.float32))}


def _snap(w):
    return [x.clone() for x in (w.act_rec, w.logp, w.value, w.h_hist, w.c_hist)]


@pytest.mark.parametrize("lengths", [None, [6, 5, 3, 2]], ids=["equal", "ragged"])
def test_graph_replays_match_eager(P, lengths):
    from paper_1911_00357_amd.worker import Worker
    say(f"graph replay lengths={lengths}")
    net, T, N = MINI_RESNET, 6, 4
    w = Worker(net, "f32", T, N, R.init_params(net, 3, random_affine=True), device="cuda")
    env = _env(net, T, N, 4, "cuda")
    w.collect(env, lengths)
    torch.cuda.synchronize()
    ref = _snap(w)
    other = _env(net, T, N, 5, "cuda")
    for rep in range(3):
        for x in (w.act_rec, w.logp, w.value, w.h_hist, w.c_hist):
            if x is not w.act_rec and x is not w.h_hist and x is not w.c_hist:
                x.zero_()
        w.collect(env, lengths, graph=True)
        torch.cuda.synchronize()
        got = _snap(w)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), rep
        w.collect(other, lengths)      # eager work between replays
        torch.cuda.synchronize()


def test_library_graph_on_a_side_stream_and_per_step(P):
    """The library's act graphs: one per argument set (count checked), each
    launched on the caller's current stream (a side stream here, with the
    results read on that stream before any synchronisation), and the
    per-step graphs of a rollout run one step at a time equal to the whole
    rollout's graph."""
    from paper_1911_00357_amd.worker import Worker
    say("library act graphs: side stream, per-step graphs")
    net, T, N = MINI_RESNET, 5, 3
    w = Worker(net, "f32", T, N, R.init_params(net, 4, random_affine=True), device="cuda")
    env = _env(net, T, N, 6, "cuda")
    w.collect(env)
    torch.cuda.synchronize()
    ref = _snap(w)
    assert w.net.graph_count() == 0
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for rep in range(3):
            w.logp.zero_()
            w.value.fill_(7.0)
            w.collect(env, graph=True)            # captured on the first call, launched after
            got = [x.clone() for x in _snap(w)]   # ordered after the graph on the same stream
            side.synchronize()
            for a, b in zip(got, ref):
                assert torch.equal(a, b), rep
    assert w.net.graph_count() == 1
    io = w._rollout_io(env)
    for rep in range(2):
        w.logp.zero_()
        w.value.zero_()
        for t in range(T + 1):
            w.net.collect(io, w.params, None, steps=(t, t + 1), graph=True)
        torch.cuda.synchronize()
        for a, b in zip(_snap(w), ref):
            assert torch.equal(a, b), rep
    assert w.net.graph_count() == 1 + (T + 1)
    assert w.net.clear_graphs() == T + 2 and w.net.graph_count() == 0
    w.release()


def test_library_graph_trim_mode_per_length_set(P):
    """ppo_collect with trim (each step launched on its active rows only,
    host lengths in the graph's key): a graph per set of lengths, each
    launch bit for bit the eager trimmed loop, the same lengths again
    reusing their graph."""
    from paper_1911_00357_amd.worker import Worker
    say("library act graphs, trim mode")
    net, T, N = MINI_RESNET, 6, 4
    w = Worker(net, "f32", T, N, R.init_params(net, 5, random_affine=True), device="cuda")
    env = _env(net, T, N, 7, "cuda")
    sets = ([6, 5, 3, 2], [6, 6, 1, 1], [6, 5, 3, 2])
    for k, lens in enumerate(sets):
        w.collect(env, lens, trim=True)           # eager
        torch.cuda.synchronize()
        ref = _snap(w)
        for rep in range(2):
            w.logp.zero_()
            w.value.zero_()
            w.collect(env, lens, trim=True, graph=True)
            torch.cuda.synchronize()
            got = _snap(w)
            # rows past an env's length are not written in trim mode: compare the written ones
            for t in range(T + 1):
                rows = sum(1 for x in lens if x >= t)
                assert torch.equal(got[1][t, :rows], ref[1][t, :rows]), (lens, rep, t)
                assert torch.equal(got[2][t, :rows], ref[2][t, :rows]), (lens, rep, t)
                assert torch.equal(got[0][t + 1, :rows], ref[0][t + 1, :rows]), (lens, rep, t)
        assert w.net.graph_count() == min(k + 1, 2)   # the third set repeats the first
    w.release()
