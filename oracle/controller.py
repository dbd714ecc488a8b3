"""The neural-controller transfer system, in float64 (Sec. 6 "Transfer
Learning", the neural controller; appendix "Neural controller additional
details").  Test infrastructure: the slow reference the GPU path is checked
against; nothing on the product path imports it.

A trained PointGoal agent is frozen and used as a closed-loop controller.
Its visual encoder's features of each frame feed two recurrent cores:

  planner     the agent's policy layout (visual FC + ReLU, previous-action
              embedding with the start token, 2-layer LSTM), with a 512-d
              hidden state and no goal input; its head gives a value and a
              raw 3-vector r, turned into a PointGoal in magnitude / unit
              direction form: g = [ELU(r0) + 0.75, tanh(r1), tanh(r2)] (the
              direction is not renormalised);
  controller  the frozen agent's own core, whose goal FC reads g in place of
              the [d, cos theta, sin theta] of a sensed goal; its head gives
              the action distribution.

PPO (Eq. 2 with the value and entropy terms, weights of Sec. 3) uses the
controller's log-probabilities and the planner's value; only the planner is
trained: the gradient reaches it through the frozen controller core (the
controller's and the encoder's parameters get none).

The three parts are separate nets of the flat format: the encoder is the
full agent (its 'enc.*' tensors are used), the controller core is a
features-in net (trunk 'none', goal mode 'vec3') whose parameters are the
agent's after its encoder (the flat format puts the encoder first), and the
planner is a features-in net with goal mode 'none' and 3 head outputs.
"""
from __future__ import annotations

import numpy as np

from . import nn, params, policy
from . import ppo as oppo


def elu(x):
    """ELU with alpha 1: x for x > 0, exp(x) - 1 otherwise."""
    return np.where(x > 0, x, np.expm1(np.minimum(x, 0.0)))


def goal_transform(raw):
    """Planner head outputs [.., 3] -> PointGoal [magnitude, direction]."""
    raw = np.asarray(raw, np.float64)
    return np.stack([elu(raw[..., 0]) + 0.75, np.tanh(raw[..., 1]), np.tanh(raw[..., 2])], axis=-1)


def goal_transform_backward(raw, dgoal):
    """d/d raw of goal_transform, given d/d goal."""
    raw = np.asarray(raw, np.float64)
    d0 = dgoal[..., 0] * np.where(raw[..., 0] > 0, 1.0, np.exp(np.minimum(raw[..., 0], 0.0)))
    d1 = dgoal[..., 1] * (1.0 - np.tanh(raw[..., 1]) ** 2)
    d2 = dgoal[..., 2] * (1.0 - np.tanh(raw[..., 2]) ** 2)
    return np.stack([d0, d1, d2], axis=-1)


def features(agent_net, agent_flat, obs, quant=None):
    """The frozen encoder's features of frames [F, C, H, W] -> [F, flat]
    (quant: the precision form of oracle.policy)."""
    P = policy.quantize_params(agent_net, params.unpack(agent_net, agent_flat), quant)
    return policy.encode(P, agent_net, obs, quant=quant)


def _cores(sys, quant):
    Pp = policy.quantize_params(sys.plan_net, params.unpack(sys.plan_net, sys.plan_flat), quant)
    Pc = policy.quantize_params(sys.ctrl_net, params.unpack(sys.ctrl_net, sys.ctrl_flat), quant)
    return Pp, Pc


def act(sys, obs, prev_a, mask, hp, cp, hc, cc, u, feat=None, quant=None):
    """One act step of the system for B envs: features, planner step, goal,
    controller step, inverse-CDF sample.  hp/cp and hc/cc: the planner's and
    the controller's [L, B, H] states.  feat [B, flat]: given features (else
    the encoder's of obs); quant: the precision form of oracle.policy for
    every product operand.  Returns a dict: action, logp (the controller's),
    value (the planner's), goal [B, 3], raw [B, 3], logits, and the next
    states."""
    if feat is None:
        feat = features(sys.agent_net, sys.agent_flat, obs, quant)
    feat = np.asarray(feat, np.float64)[None]
    Pp, Pc = _cores(sys, quant)
    m = np.asarray(mask, np.float64)[None]
    pa = np.asarray(prev_a)[None]
    raw, value, (hp2, cp2), _ = policy.core_forward(Pp, sys.plan_net, feat, None, pa, m, hp, cp, quant=quant)
    goal = goal_transform(raw[0])
    logits, _, (hc2, cc2), _ = policy.core_forward(Pc, sys.ctrl_net, feat, goal[None], pa, m, hc, cc, quant=quant)
    lp = nn.log_softmax(logits[0])
    a = policy.sample(lp, u)
    return {"action": a, "logp": np.take_along_axis(lp, a[:, None], axis=1)[:, 0], "value": value[0],
            "goal": goal, "raw": raw[0], "logits": logits[0], "hp": hp2, "cp": cp2, "hc": hc2, "cc": cc2}


def loss_grad(sys, ppo_cfg, mb, with_grad=True, adv_norm=None, feat=None, quant=None):
    """PPO loss of one minibatch of the system and its gradient with respect
    to the planner's flat parameters.  mb as oppo.minibatch_inputs gives it
    (frames 'obs', 'prev_action', 'mask', 'action', 'logp_old', 'adv', 'ret',
    'lens'), with the controller's start state 'h0', 'c0' and the planner's
    'h0_plan', 'c0_plan' [L, B, H].  feat [T_B, B, flat]: given features of
    the frames (else the encoder's); quant: the precision form of
    oracle.policy (every product operand of the encoder and the two cores
    rounded; straight-through gradients).  Returns (stats [8], planner
    gradient or None, extras) with extras holding the planner's raw outputs,
    the goals and the controller's logits [T_B, B, .]."""
    lens = mb["lens"]
    TB, B = mb["action"].shape
    valid = np.arange(TB)[:, None] < lens[None, :]
    tt, jj = np.nonzero(valid)
    if feat is None:
        feat = np.zeros((TB, B, sys.ctrl_net.flat_dim))
        feat[tt, jj] = features(sys.agent_net, sys.agent_flat, mb["obs"][tt, jj], quant)
    feat = np.where(valid[..., None], np.asarray(feat, np.float64), 0.0)
    Pp, Pc = _cores(sys, quant)
    raw, values, _, tape_p = policy.core_forward(Pp, sys.plan_net, feat, None, mb["prev_action"], mb["mask"],
                                                 mb["h0_plan"], mb["c0_plan"], keep=with_grad, quant=quant)
    goal = goal_transform(raw)
    logits, _, _, tape_c = policy.core_forward(Pc, sys.ctrl_net, feat, goal, mb["prev_action"], mb["mask"],
                                               mb["h0"], mb["c0"], keep=with_grad, quant=quant)
    stats, dlogits, dvalues = oppo.objective(logits, values, mb, ppo_cfg, adv_norm, with_grad)
    extras = {"raw": raw, "goal": goal, "logits": logits, "values": values}
    if not with_grad:
        return stats, None, extras
    # frozen controller: its parameter gradients are discarded, its goal-input gradient kept
    dgoal = np.zeros((TB, B, 3))
    policy.core_backward(Pc, sys.ctrl_net, tape_c, dlogits, np.zeros_like(values), {}, dgoal=dgoal)
    draw = goal_transform_backward(raw, dgoal)
    grads = {}
    policy.core_backward(Pp, sys.plan_net, tape_p, draw, dvalues, grads)
    extras.update({"dlogits": dlogits, "dvalues": dvalues, "dgoal": dgoal, "draw": draw})
    return stats, params.pack(sys.plan_net, grads), extras
