"""The neural-controller transfer system on the GPU (Sec. 6 "Transfer
Learning"; appendix "Neural controller additional details").

A trained PointGoal agent is frozen and used as a closed-loop controller; a
planner with the agent's policy layout (no goal input, 512-d by default)
reads the frozen encoder's features and the previous action, and its head
gives a value and a raw 3-vector that ppo_planner_goal turns into a
PointGoal [ELU(r0) + 0.75, tanh(r1), tanh(r2)] for the controller's goal FC.
PPO uses the controller's log-probabilities and the planner's value, and
only the planner is trained: its gradient comes back through the frozen
controller core (ppo_policy_backward_ex with no parameter gradient, giving
the goal-input gradient) and the transform's derivative.

Host-side sequencing only; every numeric step is a library call.  The
agent's flat parameters serve both the encoder (the full agent net, through
ppo_encode) and the controller core (a features-in net whose flat format is
the agent's after its encoder tensors: a view, nothing copied).
"""
from __future__ import annotations

from dataclasses import replace

import torch

from .api import Net, cast_bf16, planner_goal, planner_goal_backward


def controller_specs(agent, plan_hidden: int = 512):
    """(controller core, planner) network descriptions built on an agent's:
    both read the agent's flattened encoder features (trunk 'none'); the
    controller core keeps the agent's policy and reads a given 3-vector goal;
    the planner has a plan_hidden-wide visual FC and LSTM, the agent's
    previous actions, no goal input and 3 head outputs besides the value."""
    if agent.goal_mode != "polar":
        raise ValueError("the controller's goal FC must read a 3-vector (polar goal agents)")
    feat = dict(trunk="none", in_ch=agent.flat_dim, in_hw=1, avgpool=False)
    ctrl = replace(agent, goal_mode="vec3", **feat)
    plan = replace(agent, goal_mode="none", goal_dim=0, num_actions=3, prev_actions=agent.num_actions,
                   hidden=plan_hidden, vis_hidden=plan_hidden, **feat)
    return ctrl, plan


class NeuralController:
    def __init__(self, agent_spec, agent_params, plan_params, dtype: str = "f32", plan_hidden: int = 512,
                 device="cuda"):
        self.dev = torch.device(device)
        self.bf16 = dtype == "bf16"
        self.enc = Net(agent_spec, dtype)
        ctrl_spec, plan_spec = controller_specs(agent_spec, plan_hidden)
        self.ctrl, self.plan = Net(ctrl_spec, dtype), Net(plan_spec, dtype)
        enc_end = next(off for name, off, _ in self.enc.tensors() if name == "fc.w")
        self.agent = torch.as_tensor(agent_params, dtype=torch.float32).to(self.dev).contiguous()
        self.agent_lp = cast_bf16(self.agent) if self.bf16 else None
        assert self.agent.numel() == self.enc.P and self.agent.numel() - enc_end == self.ctrl.P
        # the frozen controller core: the agent's parameters after its encoder (views)
        self.ctrl_params = self.agent[enc_end:]
        self.ctrl_lp = self.agent_lp[enc_end:] if self.bf16 else None
        self.plan_params = torch.as_tensor(plan_params, dtype=torch.float32).to(self.dev).contiguous()
        assert self.plan_params.numel() == self.plan.P
        self.plan_lp = cast_bf16(self.plan_params) if self.bf16 else None

    def refresh_planner_copy(self):
        """Re-cast the planner's bfloat16 working copy after its master weights changed."""
        if self.bf16:
            self.plan_lp = cast_bf16(self.plan_params)

    def features(self, obs, out=None):
        """The frozen encoder's features [B, flat] of frames obs [B, C, H, W]."""
        return self.enc.encode(obs, self.agent, self.agent_lp, out=out)

    def act(self, obs, prev_action, mask, hp, cp, hc, cc, u, feat_out=None):
        """One act step for B envs: features, planner step, PointGoal,
        controller step and sample.  hp/cp, hc/cc: the planner's and the
        controller's [L, B, H] states (read, and the next ones returned).
        feat_out (optional [B, flat]): where the features are kept (the
        learner reuses them)."""
        feat = self.features(obs, out=feat_out)
        p = self.plan.act(feat, None, prev_action, mask, hp, cp, u, self.plan_params, self.plan_lp,
                          want_logits=True)
        goal = planner_goal(p["logits"])
        c = self.ctrl.act(feat, goal, prev_action, mask, hc, cc, u, self.ctrl_params, self.ctrl_lp,
                          want_logits=True)
        return {"action": c["action"], "logp": c["logp"], "value": p["value"], "goal": goal,
                "raw": p["logits"], "logits": c["logits"], "hp": p["h"], "cp": p["c"], "hc": c["h"],
                "cc": c["c"], "feat": feat}

    def loss_backward(self, ro, env_ids, lengths, cfg=None, loss_scale=None, adv_stats=None, grad=None):
        """One minibatch of whole env sequences: the PPO loss on the
        controller's log-probabilities and the planner's value, and S*dL/d
        (planner parameters).  ro: 'feat' [T+1, N, flat] (the frozen features),
        'prev_action', 'action' [T+1, N] int32, 'mask', 'logp' [T+1, N],
        'adv', 'ret' [T, N], the controller's start state 'h0', 'c0' and the
        planner's 'h0_plan', 'c0_plan' [L, N, H].  Returns (grad, stats [8])."""
        T1, N = ro["mask"].shape
        plan_ro = {k: ro[k] for k in ("mask", "prev_action")}
        plan_ro.update(obs=ro["feat"], h0=ro["h0_plan"], c0=ro["c0_plan"])
        raw, values, src = self.plan.policy_forward(plan_ro, env_ids, lengths, self.plan_params, self.plan_lp)
        goal = planner_goal(raw, dst=src, rows=T1 * N).view(T1, N, 3)
        ctrl_ro = dict(ro)
        ctrl_ro.update(obs=ro["feat"], goal=goal)
        logits, _, _ = self.ctrl.policy_forward(ctrl_ro, env_ids, lengths, self.ctrl_params, self.ctrl_lp)
        dlogits, dvalues, stats, _ = self.ctrl.loss_head(ctrl_ro, env_ids, lengths, logits, values, cfg,
                                                         loss_scale, adv_stats)
        F = raw.shape[0]
        dgoal = torch.empty(F, 3, dtype=torch.float32, device=raw.device)
        self.ctrl.policy_backward_ex(ctrl_ro, env_ids, lengths, self.ctrl_params, self.ctrl_lp, dlogits,
                                     torch.zeros_like(dvalues), grad=None, dgoal=dgoal)
        draw = planner_goal_backward(raw, dgoal)
        grad = self.plan.policy_backward(plan_ro, env_ids, lengths, self.plan_params, self.plan_lp, draw, dvalues,
                                         grad)
        return grad, stats
