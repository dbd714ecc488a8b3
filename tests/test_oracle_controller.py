"""Pins for the oracle's neural-controller system (Sec. 6 "Transfer
Learning"; appendix "Neural controller additional details"): the goal
transform against its closed forms and torch's ELU / tanh with autograd; the
whole system's PPO loss and planner gradient against an independent torch
float64 model with autograd (controller and encoder frozen); central finite
differences of the planner gradient; and the frozen parts receiving no
gradient while the goal path carries one."""

import numpy as np
import torch
import torch.nn.functional as F

from oracle import controller as OC
from oracle import params
from synth import rollout as R
from synth.configs import controller_nets
from tests import torch_ref
from tests.nets import MINI_RESNET, wl
from tests.test_oracle_policy import random_minibatch


class System:
    def __init__(self, agent, agent_flat, plan_hidden, plan_seed):
        self.agent_net, self.agent_flat = agent, np.asarray(agent_flat, np.float64)
        self.ctrl_net, self.plan_net = controller_nets(agent, plan_hidden)
        enc = params.offsets(agent)["fc.w"][0]          # the encoder's tensors come first
        self.ctrl_flat = self.agent_flat[enc:]
        self.plan_flat = R.init_params(self.plan_net, plan_seed, random_affine=True).astype(np.float64)


def _system(seed=1, plan_hidden=12):
    agent = MINI_RESNET
    return System(agent, R.init_params(agent, seed, random_affine=True), plan_hidden, seed + 50)


def _mb(sys, T=4, B=3, seed=5):
    mb = random_minibatch(sys.agent_net, T, B, seed)
    g = np.random.default_rng(seed + 1)
    L, H = sys.plan_net.lstm_layers, sys.plan_net.hidden
    mb["h0_plan"] = 0.5 * g.standard_normal((L, B, H))
    mb["c0_plan"] = 0.5 * g.standard_normal((L, B, H))
    return mb


def test_goal_transform_closed_forms_and_torch():
    raw = np.array([[0.0, 0.0, 0.0], [3.0, 20.0, -20.0], [-30.0, 0.5, -0.5], [1e-3, -1e-3, 2.0]])
    g = OC.goal_transform(raw)
    np.testing.assert_array_equal(g[0], [0.75, 0.0, 0.0])             # ELU(0) + 0.75, tanh(0)
    assert g[1, 0] == 3.75 and g[1, 1] == 1.0 and g[1, 2] == -1.0      # identity for x > 0; tanh saturates
    assert abs(g[2, 0] - (-0.25)) < 1e-12                             # ELU -> -1 for x << 0
    np.testing.assert_allclose(g[2, 1:], [np.tanh(0.5), -np.tanh(0.5)], rtol=0, atol=0)
    r = np.random.default_rng(0).standard_normal((5, 7, 3)) * 2
    rt = torch.tensor(r, requires_grad=True)
    gt = torch.stack([F.elu(rt[..., 0]) + 0.75, torch.tanh(rt[..., 1]), torch.tanh(rt[..., 2])], -1)
    np.testing.assert_allclose(OC.goal_transform(r), gt.detach().numpy(), rtol=1e-14, atol=1e-15)
    d = np.random.default_rng(1).standard_normal(r.shape)
    gt.backward(torch.tensor(d))
    np.testing.assert_allclose(OC.goal_transform_backward(r, d), rt.grad.numpy(), rtol=1e-13, atol=1e-15)
    # the ELU's derivative is continuous at 0 (1 from both sides)
    h = 1e-7
    fd = (OC.goal_transform(np.array([h, 0, 0]))[0] - OC.goal_transform(np.array([-h, 0, 0]))[0]) / (2 * h)
    assert abs(fd - 1.0) < 1e-6


def test_controller_nets_share_the_agent_core_layout():
    """The controller core reads the agent's parameters after its encoder:
    same names, shapes and relative offsets."""
    sysm = _system()
    oa, oc = params.offsets(sysm.agent_net), params.offsets(sysm.ctrl_net)
    enc = oa["fc.w"][0]
    assert list(oc) == [k for k in oa if oa[k][0] >= enc]
    for k, (off, shp) in oc.items():
        assert oa[k] == (off + enc, shp)
    assert params.count(sysm.ctrl_net) == sysm.ctrl_flat.size
    # the planner: no goal input, 3 outputs + value, the agent's previous actions (+ start token)
    P = params.unpack(sysm.plan_net, sysm.plan_flat)
    assert P["head.w"].shape[0] == 4 and "goal.w" not in P
    assert P["emb"].shape[0] == sysm.agent_net.num_actions + 1


def test_system_loss_and_planner_gradient_vs_torch_autograd():
    sysm = _system()
    mb = _mb(sysm)
    p = wl(sysm.agent_net).ppo
    stats, g, ex = OC.loss_grad(sysm, p, mb)
    L_t, g_t, goal_t = torch_ref.controller_system_loss(sysm.agent_net, sysm.agent_flat, sysm.ctrl_net,
                                                        sysm.ctrl_flat, sysm.plan_net, sysm.plan_flat, p, mb)
    assert abs(stats[0] - L_t) <= 1e-11 * max(1.0, abs(L_t))
    assert np.linalg.norm(g - g_t) / np.linalg.norm(g_t) < 1e-10
    lens = mb["lens"]
    valid = np.arange(mb["action"].shape[0])[:, None] < lens[None, :]
    np.testing.assert_allclose(ex["goal"][valid], goal_t[valid], rtol=1e-12, atol=1e-13)
    # the goal path carries gradient (the planner is trained through the controller)
    assert np.abs(ex["dgoal"][valid]).max() > 0
    Pg = params.unpack(sysm.plan_net, g)
    assert np.abs(Pg["lstm0.w"]).max() > 0 and np.abs(Pg["fc.w"]).max() > 0


def test_planner_gradient_central_finite_differences():
    sysm = _system(seed=3)
    mb = _mb(sysm, seed=9)
    p = wl(sysm.agent_net).ppo
    _, g, _ = OC.loss_grad(sysm, p, mb)
    base = sysm.plan_flat.copy()

    def f(th):
        sysm.plan_flat = th
        return OC.loss_grad(sysm, p, mb, with_grad=False)[0][0]

    rng = np.random.default_rng(4)
    try:
        for _ in range(5):
            d = rng.standard_normal(base.size)
            d /= np.linalg.norm(d)
            fd = (f(base + 1e-6 * d) - f(base - 1e-6 * d)) / 2e-6
            assert abs(fd - g @ d) <= 1e-6 * max(abs(fd), 1e-4), (fd, g @ d)
    finally:
        sysm.plan_flat = base


def test_frozen_controller_and_constant_goal():
    """With the planner's goal head zeroed (weights and bias 0 on the three
    goal rows) every goal is [0.75, 0, 0]: the controller then sees a fixed
    PointGoal and its logits equal the agent core run on that goal."""
    from oracle import policy
    sysm = _system(seed=6)
    P = params.unpack(sysm.plan_net, sysm.plan_flat)
    P["head.w"][:3] = 0.0
    P["head.b"][:3] = 0.0
    sysm.plan_flat = params.pack(sysm.plan_net, P)
    mb = _mb(sysm, seed=13)
    _, _, ex = OC.loss_grad(sysm, wl(sysm.agent_net).ppo, mb, with_grad=False)
    TB, B = mb["action"].shape
    lens = mb["lens"]
    valid = np.arange(TB)[:, None] < lens[None, :]
    np.testing.assert_array_equal(ex["goal"][valid], np.broadcast_to([0.75, 0.0, 0.0], (valid.sum(), 3)))
    tt, jj = np.nonzero(valid)
    feat = np.zeros((TB, B, sysm.ctrl_net.flat_dim))
    feat[tt, jj] = OC.features(sysm.agent_net, sysm.agent_flat, mb["obs"][tt, jj])
    Pc = params.unpack(sysm.ctrl_net, sysm.ctrl_flat)
    logits, _, _, _ = policy.core_forward(Pc, sysm.ctrl_net, feat, np.broadcast_to([0.75, 0.0, 0.0], (TB, B, 3)),
                                          mb["prev_action"], mb["mask"], mb["h0"], mb["c0"])
    np.testing.assert_array_equal(ex["logits"], logits)


def test_system_act_step_matches_the_learner_forward():
    """One act step equals the first frame of the learner's forward on the
    same inputs (the rollout and the learner compute the same policy)."""
    sysm = _system(seed=8)
    mb = _mb(sysm, T=1, B=3, seed=17)
    mb["lens"] = np.full(3, 1)
    u = np.random.default_rng(2).random(3)
    out = OC.act(sysm, mb["obs"][0], mb["prev_action"][0], mb["mask"][0], mb["h0_plan"], mb["c0_plan"],
                 mb["h0"], mb["c0"], u)
    _, _, ex = OC.loss_grad(sysm, wl(sysm.agent_net).ppo, mb, with_grad=False)
    np.testing.assert_allclose(out["goal"], ex["goal"][0], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(out["logits"], ex["logits"][0], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(out["value"], ex["values"][0], rtol=1e-13, atol=1e-14)


def test_given_features_and_precision_form():
    """The learner with the encoder's own features passed in equals the
    default; the bfloat16 precision form moves the loss at bfloat16 scale."""
    sysm = _system(seed=11)
    mb = _mb(sysm, seed=21)
    p = wl(sysm.agent_net).ppo
    s0, g0, _ = OC.loss_grad(sysm, p, mb)
    TB, B = mb["action"].shape
    feat = OC.features(sysm.agent_net, sysm.agent_flat, mb["obs"].reshape(TB * B, *mb["obs"].shape[2:]))
    s1, g1, _ = OC.loss_grad(sysm, p, mb, feat=feat.reshape(TB, B, -1))
    np.testing.assert_array_equal(s0, s1)
    np.testing.assert_array_equal(g0, g1)
    sq, gq, _ = OC.loss_grad(sysm, p, mb, quant="bf16")
    assert 1e-6 < abs(sq[0] - s0[0]) / abs(s0[0]) < 1e-1
    assert 1e-6 < np.linalg.norm(gq - g0) / np.linalg.norm(g0) < 2e-1
