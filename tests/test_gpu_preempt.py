"""Rollouts whose envs stop at different steps (Sec. 3, preemption) on the
GPU: ppo_act's device row count, one captured graph serving any lengths, and
a worker whose rollout the preemption monitor ends early.

The row count only decides which rows are written; rows are independent, so
the written rows must equal those of a call without it bit for bit, and every
other row must keep what it held.  The preempted rollout must be the prefix
of the full one (same kernels on the same inputs, bit for bit) and end at the
step the monitor's rule gives for the scripted finished counts."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import ppo
from synth import rollout as R
from tests.gpu_util import assert_close
from tests.nets import MINI_RESNET, TINY_NET
from tests.test_gpu_parity import say
from tests.test_gpu_graph import _env

pytestmark = pytest.mark.gpu


def _act_inputs(net, B, L, H, seed, dev="cuda"):
    g = np.random.default_rng(seed)
    t = lambda a: torch.as_tensor(a).to(dev)
    return dict(obs=t(g.random((B, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32)),
                goal=t(g.standard_normal((B, 2)).astype(np.float32)),
                prev_action=t(g.integers(0, 4, B).astype(np.int32)),
                mask=t((g.random(B) > 0.3).astype(np.float32)),
                h_in=t(g.standard_normal((L, B, H)).astype(np.float32)),
                c_in=t(g.standard_normal((L, B, H)).astype(np.float32)),
                u=t(g.random(B).astype(np.float32)))


def _outs(B, L, H, A, fill):
    f = dict(dtype=torch.float32, device="cuda")
    return {"action": torch.full((B,), -7, dtype=torch.int32, device="cuda"),
            "logp": torch.full((B,), fill, **f), "value": torch.full((B,), fill, **f),
            "h": torch.full((L, B, H), fill, **f), "c": torch.full((L, B, H), fill, **f),
            "logits": torch.full((B, A), fill, **f)}


# tiny_3layer: a core of three LSTM layers, run by the per-layer step kernel
# (h and c written to workspace rows, then the active rows copied out)
NETS = {"tiny": TINY_NET, "mini_resnet": MINI_RESNET, "tiny_3layer": dataclasses.replace(TINY_NET, lstm_layers=3)}


@pytest.mark.parametrize("netname", list(NETS))
def test_act_row_count(P, netname):
    net = NETS[netname]
    B = 5
    n = P.Net(net, "f32")
    L, H, A = net.lstm_layers, net.hidden, net.num_actions
    params = torch.tensor(R.init_params(net, 1, random_affine=True), device="cuda")
    x = _act_inputs(net, B, L, H, 2)
    full = n.act(x["obs"], x["goal"], x["prev_action"], x["mask"], x["h_in"], x["c_in"], x["u"], params,
                 out=_outs(B, L, H, A, 0.0))
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    for k in (0, 2, 5, 9, -3):
        say(f"act row count {netname}: {k} of {B}")
        kk = min(max(k, 0), B)
        cnt.fill_(k)
        o = n.act(x["obs"], x["goal"], x["prev_action"], x["mask"], x["h_in"], x["c_in"], x["u"], params,
                  out=_outs(B, L, H, A, 123.0), active=cnt)
        torch.cuda.synchronize()
        for key in ("action", "logp", "value", "logits"):
            assert torch.equal(o[key][:kk], full[key][:kk]), key
        for key in ("h", "c"):
            assert torch.equal(o[key][:, :kk], full[key][:, :kk]), key
            assert torch.all(o[key][:, kk:] == 123.0), key
        assert torch.all(o["action"][kk:] == -7)
        for key in ("logp", "value", "logits"):
            assert torch.all(o[key][kk:] == 123.0), key
    # the state updated in place: rows past the count keep their state
    cnt.fill_(3)
    h, c = x["h_in"].clone(), x["c_in"].clone()
    o = _outs(B, L, H, A, 0.0)
    o["h"], o["c"] = h, c
    n.act(x["obs"], x["goal"], x["prev_action"], x["mask"], h, c, x["u"], params, out=o, active=cnt)
    torch.cuda.synchronize()
    assert torch.equal(h[:, :3], full["h"][:, :3]) and torch.equal(h[:, 3:], x["h_in"][:, 3:])
    assert torch.equal(c[:, :3], full["c"][:, :3]) and torch.equal(c[:, 3:], x["c_in"][:, 3:])


def _snap(w, T, lens):
    """The written part of a rollout: per env n, steps t <= T_n."""
    out = {}
    for nm, x in (("action", w.act_rec[1:]), ("logp", w.logp), ("value", w.value)):
        out[nm] = [x[:lens[i] + 1, i].clone() for i in range(len(lens))]
    out["h"] = [w.h_hist[:min(lens[i] + 1, T) + 1, :, i].clone() for i in range(len(lens))]
    return out


def _same(a, b, tol=None):
    for k in a:
        for x, y in zip(a[k], b[k]):
            if tol is None:
                assert torch.equal(x, y), k
            else:
                assert_close(k, x.cpu().numpy(), y.cpu().numpy().astype(np.float64), tol)


def test_one_graph_serves_any_lengths(P):
    from paper_1911_00357_amd.worker import Worker
    net, T, N = MINI_RESNET, 6, 4
    w = Worker(net, "f32", T, N, R.init_params(net, 3, random_affine=True), device="cuda")
    env = _env(net, T, N, 4, "cuda")
    for k, lens in enumerate(([6, 5, 3, 2], [6, 6, 6, 6], [4, 4, 1, 1], [2, 2, 2, 2])):
        say(f"one graph, lengths {lens}")
        w.collect(env, lens)                        # eager, device row counts
        torch.cuda.synchronize()
        eager = _snap(w, T, lens)
        w.collect(env, lens, trim=True)             # eager, each step on its active rows only
        torch.cuda.synchronize()
        trimmed = _snap(w, T, lens)
        w.logp.zero_()
        w.value.zero_()
        w.collect(env, lens, graph=True)
        torch.cuda.synchronize()
        assert w.net.graph_count() == 1             # the library's graph of these buffers
        got = _snap(w, T, lens)
        _same(got, eager)
        # fewer rows: other GEMM shapes, so equal to float32 rounding only
        for nm in ("logp", "value", "h"):
            _same({nm: got[nm]}, {nm: trimmed[nm]}, 1e-5)
        assert all(torch.equal(x, y) for x, y in zip(got["action"], trimmed["action"]))


class ScriptedStore:
    """A key-value store whose finished count for the other workers jumps to
    `others` at the `at`-th query (a stand-in for the shared TCPStore);
    this worker's own completion is added on top."""

    def __init__(self, others, at):
        self.others, self.at, self.queries, self.own = others, at, 0, 0

    def add(self, key, n):
        if n == 0:
            self.queries += 1
        self.own += n
        return self.own + (self.others if self.queries >= self.at else 0)


@pytest.mark.parametrize("at", [1, 3, 100], ids=["at_floor", "mid", "never"])
def test_preempted_rollout(P, at):
    from paper_1911_00357_amd.preempt import PreemptionMonitor, collect as run_steps
    from paper_1911_00357_amd.worker import PPOHyper, Worker
    net, T, N, W = MINI_RESNET, 12, 4, 5
    # the step the monitor's rule ends the rollout at, on the host alone
    expect = run_steps(PreemptionMonitor(ScriptedStore(W - 1, at), W, T), 0, lambda t: None)
    say(f"preempted rollout: finished count at query {at}: T_w = {expect} of {T}")
    hp = PPOHyper(epochs=1, minibatches=2)
    w = Worker(net, "f32", T, N, R.init_params(net, 3, random_affine=True), hp, device="cuda")
    env = _env(net, T, N, 4, "cuda")
    w.collect(env, None, graph=True)                 # the full rollout, one graph
    torch.cuda.synchronize()
    full = _snap(w, T, [T] * N)
    w.logp.zero_()
    w.value.zero_()
    Tw = w.collect(env, graph=True, monitor=PreemptionMonitor(ScriptedStore(W - 1, at), W, T))
    torch.cuda.synchronize()
    assert Tw == expect
    lens = [Tw] * N
    got = _snap(w, T, lens)
    pref = {k: [x[:len(y)] for x, y in zip(full[k], got[k])] for k in full}
    _same(got, pref)
    # the update on the cut rollout: GAE bootstraps from V[T_w] (oracle)
    g = np.random.default_rng(7)
    env["reward"] = torch.tensor(g.standard_normal((T, N)).astype(np.float32), device="cuda")
    env["done"] = torch.tensor((g.random((T, N)) < 0.1).astype(np.uint8), device="cuda")
    adv, ret = w.update(env, [[np.array([0, 1]), np.array([2, 3])]], lens)
    torch.cuda.synchronize()
    A, Rt = ppo.gae(env["reward"].cpu().numpy(), w.value.cpu().numpy(), env["done"].cpu().numpy(),
                    np.array(lens), 0.99, 0.95)
    assert_close("advantages", adv.cpu().numpy(), A, 1e-5)
    assert_close("returns", ret.cpu().numpy(), Rt, 1e-5)
    assert np.isfinite(w.stats.cpu().numpy()).all() and w.adam.state()["step"] == 2
