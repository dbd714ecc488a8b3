"""Pins for the oracle's agent: the paper's stated shapes, the forward and
the hand gradient of the PPO loss against an independent torch float64
model (library modules + autograd), and central finite differences."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import params, policy, ppo
from synth import rollout as R
from tests import torch_ref
from tests.nets import TINY_NET, TINY_PLUS, MINI_RESNET, MINI_SERESNEXT, wl

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def gold(k):
    return GOLD[k]["value"]


def random_minibatch(net, T, B, seed, ragged=True, logp_spread=0.3):
    """A minibatch with random (not rollout-consistent) old log-probs so that
    both clip branches are exercised."""
    g = np.random.default_rng(seed)
    lens = g.integers(max(1, T // 2), T + 1, B) if ragged else np.full(B, T)
    lens[0] = T
    return {
        "envs": np.arange(B), "lens": lens,
        "obs": g.random((T, B, net.in_ch, net.in_hw, net.in_hw)),
        "goal": g.standard_normal((T, B, 2)),
        "prev_action": g.integers(0, net.num_actions, (T, B)),
        "mask": (g.random((T, B)) > 0.2).astype(np.float64),
        "action": g.integers(0, net.num_actions, (T, B)),
        "logp_old": np.log(0.25) + logp_spread * g.standard_normal((T, B)),
        "adv": g.standard_normal((T, B)), "ret": g.standard_normal((T, B)),
        "h0": 0.5 * g.standard_normal((net.lstm_layers, B, net.hidden)),
        "c0": 0.5 * g.standard_normal((net.lstm_layers, B, net.hidden)),
    }


# ------------------------------------------------------------ paper facts
def test_workloads_match_paper_facts():
    n = synth.C1.net
    assert n.num_actions == gold("num_actions")
    assert n.in_hw == gold("frame_hw") and n.enc_hw == gold("encoder_hw")
    assert [n.compress_ch, n.feat_hw, n.feat_hw] == gold("compress_out")
    assert n.flat_dim == gold("flatten_dim")
    assert n.goal_dim == gold("goal_out") and n.prev_act_dim == gold("prev_action_dim")
    assert n.lstm_layers == gold("lstm_layers") and n.hidden == gold("lstm_hidden")
    p = synth.C1.ppo
    assert (p.gamma, p.lam, p.lr) == (gold("gamma"), gold("gae_tau"), gold("adam_lr"))
    assert (p.epochs, p.minibatches, p.norm_adv) == (gold("ppo_epochs"), gold("minibatches"),
                                                     gold("normalize_adv"))
    assert (synth.C1.T, synth.C1.N) == (gold("rollout_T"), gold("envs_per_worker"))
    lens = R.rollout_lengths(synth.C4, 0)
    assert lens.min() >= gold("min_rollout_frac") * synth.C4.T and lens.max() <= synth.C4.T


def test_oracle_encoder_shapes_match_paper():
    net = synth.C1.net
    P = params.unpack(net, R.init_params(net, 0))
    x = policy.prep_obs(net, np.random.default_rng(0).random((1, 4, 256, 256)))
    assert x.shape[2:] == (gold("encoder_hw"),) * 2
    tape = {}
    feat = policy.encoder_forward(P, net, x, tape)
    assert list(tape["s3.b2.out"].shape[1:]) == gold("backbone_out")
    assert feat.shape == (1, gold("flatten_dim"))


def test_param_format_readers_agree():
    """The oracle's reader and the generator's reader of the flat format
    place every tensor at the same offset."""
    for net in (TINY_NET, TINY_PLUS, MINI_RESNET, MINI_SERESNEXT, synth.C1.net, synth.C3.net, synth.C5.net):
        o = params.offsets(net)
        s = synth.tensor_list(net)
        assert params.count(net) == synth.param_count(net)
        assert [v[0] for v in o.values()] == [t.offset for t in s]
        assert [tuple(v[1]) for v in o.values()] == [t.shape for t in s]


# ----------------------------------------------- loss + gradient vs autograd
@pytest.mark.parametrize("net", [TINY_NET, TINY_PLUS, MINI_RESNET, MINI_SERESNEXT],
                         ids=["tiny", "tiny+", "mini_resnet", "mini_seresnext"])
def test_loss_and_grad_vs_torch_autograd(net):
    w = wl(net)
    flat = R.init_params(net, 1, random_affine=True).astype(np.float64)
    mb = random_minibatch(net, 5, 3, seed=2)
    stats, g = ppo.loss_grad(flat, net, w.ppo, mb)
    L_t, g_t, logits_t, values_t = torch_ref.ppo_loss(net, w.ppo, flat, mb)
    assert abs(stats[0] - L_t) <= 1e-11 * max(1.0, abs(L_t))
    rel = np.linalg.norm(g - g_t) / np.linalg.norm(g_t)
    assert rel < 1e-10, rel
    assert 0.0 < stats[4] < 1.0          # some samples clipped, some not


def test_resnet_full_width_forward_vs_torch():
    """The real-width bottleneck trunk on one 64x64 frame (1x1 map)."""
    from tests.nets import RESNET_64 as net
    flat = R.init_params(net, 3, random_affine=True).astype(np.float64)
    mb = random_minibatch(net, 2, 2, seed=4, ragged=False)
    stats, g = ppo.loss_grad(flat, net, wl(net).ppo, mb)
    L_t, g_t, _, _ = torch_ref.ppo_loss(net, wl(net).ppo, flat, mb)
    assert abs(stats[0] - L_t) <= 1e-10 * max(1.0, abs(L_t))
    assert np.linalg.norm(g - g_t) / np.linalg.norm(g_t) < 1e-9


def test_seresnext_full_width_forward_vs_torch():
    """The real-width SE-ResNeXt trunk (16 groups, reduction 16) on one 64x64
    frame, loss and gradient against the torch model."""
    from tests.nets import SERESNEXT_64 as net
    flat = R.init_params(net, 3, random_affine=True).astype(np.float64)
    mb = random_minibatch(net, 2, 2, seed=4, ragged=False)
    stats, g = ppo.loss_grad(flat, net, wl(net).ppo, mb)
    L_t, g_t, _, _ = torch_ref.ppo_loss(net, wl(net).ppo, flat, mb)
    assert abs(stats[0] - L_t) <= 1e-10 * max(1.0, abs(L_t))
    assert np.linalg.norm(g - g_t) / np.linalg.norm(g_t) < 1e-9


def test_seresnext_shapes():
    """SE-ResNeXt50 with halved widths: the same 1024 x 4 x 4 backbone output
    and 2048-d flattened feature as the ResNet, 16 groups of 4 channels in the
    first stage's 3x3, SE hidden width C/16."""
    net = synth.C5.net
    P = params.unpack(net, R.init_params(net, 0))
    assert P["s0.b0.c2"].shape == (64, 4, 3, 3) and P["s3.b0.c2"].shape == (512, 32, 3, 3)
    assert P["s0.b0.se1.w"].shape == (8, 128) and P["s3.b2.se2.w"].shape == (1024, 64)
    x = policy.prep_obs(net, np.random.default_rng(0).random((1, 4, 256, 256)))
    tape = {}
    feat = policy.encoder_forward(P, net, x, tape)
    assert list(tape["s3.b2.out"].shape[1:]) == gold("backbone_out")
    assert feat.shape == (1, gold("flatten_dim"))


# ------------------------------------------------------ finite differences
@pytest.mark.parametrize("net,seed", [(TINY_PLUS, 5), (MINI_RESNET, 6), (MINI_SERESNEXT, 8)],
                         ids=["tiny+", "mini_resnet", "mini_seresnext"])
def test_grad_central_finite_differences(net, seed):
    w = wl(net)
    flat = R.init_params(net, seed, random_affine=True).astype(np.float64)
    mb = random_minibatch(net, 4, 3, seed=seed + 10)
    _, g = ppo.loss_grad(flat, net, w.ppo, mb)
    rng = np.random.default_rng(seed)
    h = 1e-6
    f = lambda th: ppo.loss_grad(th, net, w.ppo, mb, with_grad=False)[0][0]
    for _ in range(6):                                   # random directions
        d = rng.standard_normal(flat.size)
        d /= np.linalg.norm(d)            # a small step keeps clear of kinks
        fd = (f(flat + h * d) - f(flat - h * d)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(abs(fd), 1e-4), (fd, g @ d)
    for i in rng.choice(flat.size, 12, replace=False):   # single coordinates
        e = np.zeros(flat.size)
        e[i] = 1.0
        fd = (f(flat + 1e-5 * e) - f(flat - 1e-5 * e)) / 2e-5
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


# ------------------------------------------------------ act step / sampling
def test_sampling_is_inverse_cdf_brute_force():
    lp = np.log(np.array([[0.1, 0.2, 0.3, 0.4]] * 6))
    u = np.array([0.0, 0.0999, 0.1001, 0.5, 0.95, 0.999999])
    np.testing.assert_array_equal(policy.sample(lp, u), [0, 0, 1, 2, 3, 3])


def test_act_matches_torch_policy_single_step():
    net = TINY_PLUS
    flat = R.init_params(net, 7, random_affine=True).astype(np.float64)
    mb = random_minibatch(net, 1, 4, seed=8, ragged=False)
    P = params.unpack(net, flat)
    u = np.random.default_rng(1).random(4)
    out = policy.act(P, net, mb["obs"][0], mb["goal"][0], mb["prev_action"][0], mb["mask"][0],
                     mb["h0"], mb["c0"], u)
    _, tP = torch_ref.unpack(net, flat, requires_grad=False)
    import torch
    t = lambda a, dt=torch.float64: torch.tensor(np.asarray(a), dtype=dt)
    lg, vals = torch_ref.policy_seq(tP, net, t(mb["obs"]), t(mb["goal"]),
                                    t(mb["prev_action"], torch.int64), t(mb["mask"]),
                                    t(mb["h0"]), t(mb["c0"]))
    np.testing.assert_allclose(out["logits"], lg[0].numpy(), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(out["value"], vals[0].numpy(), rtol=1e-11, atol=1e-13)
    p = torch.softmax(lg[0], -1).numpy()
    brute = [min([k for k in range(4) if p[i, :k + 1].sum() > u[i]] or [3]) for i in range(4)]
    np.testing.assert_array_equal(out["action"], brute)
