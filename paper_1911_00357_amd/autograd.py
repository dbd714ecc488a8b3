"""The learner as torch.autograd.Functions over the flat parameter vector.

PolicyFunction: forward runs ppo_policy_forward (logits and values of every
frame of a minibatch of whole env sequences); backward runs
ppo_policy_backward, which recomputes the encoder and LSTM activations and
applies the hand-written backward to the incoming d(logits), d(values).

PPOLossFunction: the PPO objective (Eq. 2 with the value and entropy terms,
the per-env weights 1/(|B| T_n) of Sec. 3, the loss scale) on the policy
outputs, by ppo_loss_head: forward returns S*L and the loss statistics,
backward the library's d(S*L)/d(logits, values), times the incoming
gradient of the loss (the chain rule; 1 for a loss differentiated directly).
Together they split ppo_loss_backward in three with torch's autograd graph
in between; torch computes no part of the method.
"""
from __future__ import annotations

import torch


class PolicyFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, net, ro, env_ids, lengths, params_lp):
        logits, values, src = net.policy_forward(ro, env_ids, lengths, params, params_lp)
        ctx.net, ctx.ro, ctx.env_ids, ctx.lengths, ctx.params_lp = net, ro, env_ids, lengths, params_lp
        ctx.save_for_backward(params)
        ctx.mark_non_differentiable(src)
        return logits, values, src

    @staticmethod
    def backward(ctx, dlogits, dvalues, _dsrc):
        (params,) = ctx.saved_tensors
        dl = torch.zeros_like(dlogits) if dlogits is None else dlogits.contiguous().float()
        dv = torch.zeros_like(dvalues) if dvalues is None else dvalues.contiguous().float()
        grad = ctx.net.policy_backward(ctx.ro, ctx.env_ids, ctx.lengths, params, ctx.params_lp, dl, dv)
        return grad, None, None, None, None, None


class PPOLossFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, logits, values, net, ro, env_ids, lengths, cfg, loss_scale, adv_stats):
        dl, dv, stats, loss = net.loss_head(ro, env_ids, lengths, logits.detach().contiguous(),
                                            values.detach().contiguous(), cfg, loss_scale, adv_stats)
        ctx.save_for_backward(dl, dv)
        ctx.mark_non_differentiable(stats)
        return loss, stats

    @staticmethod
    def backward(ctx, g_loss, _g_stats):
        dl, dv = ctx.saved_tensors
        return g_loss * dl, g_loss * dv, None, None, None, None, None, None, None


def policy(params, net, ro, env_ids, lengths=None, params_lp=None):
    """(logits [F, A], values [F], frame_src [F]) with autograd support on params."""
    return PolicyFunction.apply(params, net, ro, list(env_ids), lengths, params_lp)


def ppo_loss(logits, values, net, ro, env_ids, lengths=None, cfg=None, loss_scale=None, adv_stats=None):
    """(S*L (0-dim), stats [8]) of the minibatch whose policy outputs are given
    (frames in policy()'s order), differentiable in logits and values.
    cfg: api.LossCfg (clip, coefficients, norm_adv); loss_scale: device
    float [1] (bfloat16 nets); adv_stats: device double [2] when norm_adv."""
    from .api import LossCfg
    return PPOLossFunction.apply(logits, values, net, ro, list(env_ids), lengths, cfg or LossCfg(), loss_scale,
                                 adv_stats)
