"""The policy as a torch.autograd.Function over the flat parameter vector.

forward runs ppo_policy_forward (logits and values of every frame of a
minibatch of whole env sequences); backward runs ppo_policy_backward, which
recomputes the encoder and LSTM activations and applies the hand-written
backward to the incoming d(logits), d(values).  Any loss written in torch on
the outputs (for instance the clipped surrogate of Eq. 2) can then be
differentiated with respect to the parameters.
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


def policy(params, net, ro, env_ids, lengths=None, params_lp=None):
    """(logits [F, A], values [F], frame_src [F]) with autograd support on params."""
    return PolicyFunction.apply(params, net, ro, list(env_ids), lengths, params_lp)


def ppo_loss(logits, values, src, ro, lengths_w, clip=0.2, value_coef=0.5, entropy_coef=0.01):
    """The clipped PPO loss of Eq. 2 (+ value and entropy terms) written in
    torch on the policy outputs; lengths_w [F] holds each frame's weight
    1/(|B| T_n).  Used to exercise the autograd path."""
    idx = src.long()
    a = ro["action"].reshape(-1)[idx].long()
    lp = torch.log_softmax(logits, -1)
    lpa = lp.gather(1, a[:, None])[:, 0]
    adv = ro["adv"].reshape(-1)[idx]
    ratio = torch.exp(lpa - ro["logp"].reshape(-1)[idx])
    surr = torch.min(ratio * adv, torch.clamp(ratio, 1 - clip, 1 + clip) * adv)
    ent = -(lp.exp() * lp).sum(-1)
    ret = ro["ret"].reshape(-1)[idx]
    return (-(lengths_w * surr).sum() + value_coef * (lengths_w * 0.5 * (values - ret) ** 2).sum()
            - entropy_coef * (lengths_w * ent).sum())
