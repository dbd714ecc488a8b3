"""An independent float64 PyTorch (CPU) model of the agent, built from
torch library modules, used only to pin the oracle.

It reads the flat parameter format through synth.layout (a reader separate
from the oracle's), runs conv2d / group_norm / max_pool2d / avg_pool2d /
LSTMCell / log_softmax from torch, and gets gradients from autograd.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

from synth.layout import tensor_list

GN_EPS = 1e-5


def _bf16(x):
    """Nearest bfloat16 value (ties to even) of a float64 tensor, float64."""
    m, e = torch.frexp(x)
    return torch.ldexp(torch.round(m * 256.0), (e - 8).to(x.dtype))


def quantizer(quant):
    """Operand rounding of the precision form with a straight-through
    gradient (the rounding counts as the identity for autograd)."""
    if quant is None:
        return lambda x: x
    assert quant == "bf16"
    return lambda x: x + (_bf16(x.detach()) - x.detach())


def unpack(net, flat, requires_grad=True):
    flat_t = torch.tensor(np.asarray(flat, np.float64), requires_grad=requires_grad)
    P = {}
    for t in tensor_list(net):
        n = int(np.prod(t.shape))
        a = flat_t[t.offset:t.offset + n].view(t.shape)
        if t.kind == "conv":
            a = a.permute(0, 3, 1, 2)       # O,KH,KW,I -> O,I,KH,KW
        P[t.name] = a
    return flat_t, P


def _cgn(P, net, x, conv, gn, s, p, relu, q=lambda a: a, groups=1):
    y = F.conv2d(q(x), q(P[conv]), stride=s, padding=p, groups=groups)
    y = F.group_norm(y, net.gn_groups, P[gn + ".g"], P[gn + ".b"], eps=GN_EPS)
    return F.relu(y) if relu else y


def encoder(P, net, obs, quant=None):
    q = quantizer(quant)
    cgn = lambda x, conv, gn, s, p, relu: _cgn(P, net, x, conv, gn, s, p, relu, q)
    x = obs
    if net.avgpool:
        x = F.avg_pool2d(x, 2)
    if net.trunk == "tiny":
        x = cgn(x, "enc.conv1", "enc.gn1", 2, 1, True)
        x = cgn(x, "enc.conv2", "enc.gn2", 2, 1, True)
        return x.flatten(1)
    x = cgn(x, "enc.stem", "enc.stem.gn", 2, 3, True)
    x = F.max_pool2d(x, 3, 2, 1)
    for s, nb in enumerate(net.blocks):
        for j in range(nb):
            p = f"enc.s{s}.b{j}"
            st = 2 if (j == 0 and s > 0) else 1
            se = net.trunk == "seresnext"
            y = cgn(x, p + ".c1", p + ".gn1", 1, 0, True)
            y = _cgn(P, net, y, p + ".c2", p + ".gn2", st, 1, True, q, net.cardinality if se else 1)
            y = cgn(y, p + ".c3", p + ".gn3", 1, 0, False)
            if se:     # squeeze-excite: pooled channels -> FC -> ReLU -> FC -> sigmoid gate
                z = F.adaptive_avg_pool2d(y, 1).flatten(1)
                g = torch.sigmoid(F.linear(F.relu(F.linear(z, P[p + ".se1.w"], P[p + ".se1.b"])),
                                           P[p + ".se2.w"], P[p + ".se2.b"]))
                y = y * g[:, :, None, None]
            sc = cgn(x, p + ".ds", p + ".ds.gn", st, 0, False) if j == 0 else x
            x = F.relu(y + sc)
    x = cgn(x, "enc.compress", "enc.compress.gn", 1, 1, True)
    return x.flatten(1)


def policy_seq(P, net, obs, goal, prev_a, masks, h0, c0, quant=None):
    """obs [T,B,C,H,W] -> logits [T,B,A], values [T,B].  quant: the
    precision form (every conv, visual-FC and LSTM operand rounded)."""
    T, B = obs.shape[:2]
    feat = encoder(P, net, obs.reshape(T * B, *obs.shape[2:]), quant).reshape(T, B, -1)
    return policy_core(P, net, feat, goal, prev_a, masks, h0, c0, quant)


def policy_core(P, net, feat, goal, prev_a, masks, h0, c0, quant=None):
    """feat [T,B,flat] -> logits [T,B,A], values [T,B]; goal [T,B,2] (raw or
    polar goal modes), [T,B,3] (a given 3-vector: 'vec3') or unused ('none')."""
    q = quantizer(quant)
    T, B = feat.shape[:2]
    H = net.hidden
    cells = []
    for l in range(net.lstm_layers):
        w = P[f"lstm{l}.w"]
        din = w.shape[1] - H
        cells.append((q(w[:, :din]), q(w[:, din:]), P[f"lstm{l}.b"]))
    h = [h0[l] for l in range(net.lstm_layers)]
    c = [c0[l] for l in range(net.lstm_layers)]
    logits, values = [], []
    for t in range(T):
        m = masks[t][:, None]
        v = F.relu(F.linear(q(feat[t]), q(P["fc.w"]), P["fc.b"]))
        parts = [v]
        if net.goal_mode == "polar":
            d, th = goal[t][:, 0], goal[t][:, 1]
            g3 = torch.stack([d, torch.cos(th), torch.sin(th)], 1)
            parts.append(F.linear(g3, P["goal.w"], P["goal.b"]))
        elif net.goal_mode == "vec3":
            parts.append(F.linear(goal[t], P["goal.w"], P["goal.b"]))
        elif net.goal_mode == "raw":
            parts.append(goal[t])
        if net.prev_act_dim:
            idx = torch.where(masks[t] == 0, torch.zeros_like(prev_a[t]), prev_a[t] + 1)
            parts.append(P["emb"][idx])
        x = torch.cat(parts, 1)
        for l, (wih, whh, b) in enumerate(cells):
            # torch's fused LSTM cell (gate order i, f, g, o)
            h[l], c[l] = torch._VF.lstm_cell(q(x), (q(m * h[l]), m * c[l]), wih, whh, b,
                                             torch.zeros_like(b))
            x = h[l]
        o = F.linear(x, P["head.w"], P["head.b"])
        logits.append(o[:, :net.num_actions])
        values.append(o[:, net.num_actions])
    return torch.stack(logits), torch.stack(values)


def ppo_loss(net, ppo, flat, mb, quant=None):
    """Loss of one minibatch dict (as made by oracle.ppo.minibatch_inputs),
    its gradient by autograd, and the logits/values."""
    flat_t, P = unpack(net, flat)
    tt = lambda a, dt=torch.float64: torch.tensor(np.asarray(a), dtype=dt)
    lens = tt(mb["lens"])
    TB, B = mb["action"].shape
    valid = (torch.arange(TB, dtype=torch.float64)[:, None] < lens[None, :]).double()
    w = valid / (B * lens[None, :])
    logits, values = policy_seq(P, net, tt(mb["obs"]), tt(mb["goal"]),
                                tt(mb["prev_action"], torch.int64), tt(mb["mask"]),
                                tt(mb["h0"]), tt(mb["c0"]), quant)
    lp = F.log_softmax(logits, -1)
    lpa = lp.gather(2, tt(mb["action"], torch.int64)[..., None])[..., 0]
    adv = tt(mb["adv"])
    ratio = torch.exp(lpa - tt(mb["logp_old"]))
    surr = torch.min(ratio * adv, torch.clamp(ratio, 1 - ppo.clip, 1 + ppo.clip) * adv)
    ent = -(lp.exp() * lp).sum(-1)
    L = (-(w * surr).sum() + ppo.value_coef * (w * 0.5 * (values - tt(mb["ret"])) ** 2).sum()
         - ppo.entropy_coef * (w * ent).sum())
    L.backward()
    return L.item(), flat_t.grad.numpy().copy(), logits.detach().numpy(), values.detach().numpy()


def controller_system_loss(agent_net, agent_flat, ctrl_net, ctrl_flat, plan_net, plan_flat, ppo, mb):
    """The neural-controller system's PPO loss and its gradient with respect
    to the planner's parameters only, by autograd: frozen encoder features,
    planner core -> [ELU(r0) + 0.75, tanh(r1), tanh(r2)] -> frozen controller
    core -> PPO on the controller's logits and the planner's value."""
    tt = lambda a, dt=torch.float64: torch.tensor(np.asarray(a), dtype=dt)
    lens = tt(mb["lens"])
    TB, B = mb["action"].shape
    valid = (torch.arange(TB, dtype=torch.float64)[:, None] < lens[None, :]).double()
    w = valid / (B * lens[None, :])
    _, Pa = unpack(agent_net, agent_flat, requires_grad=False)
    obs = tt(mb["obs"])
    with torch.no_grad():
        feat = encoder(Pa, agent_net, obs.reshape(TB * B, *obs.shape[2:])).reshape(TB, B, -1) * valid[..., None]
    flat_p, Pp = unpack(plan_net, plan_flat, requires_grad=True)
    _, Pc = unpack(ctrl_net, ctrl_flat, requires_grad=False)
    pa, masks = tt(mb["prev_action"], torch.int64), tt(mb["mask"])
    raw, values = policy_core(Pp, plan_net, feat, None, pa, masks, tt(mb["h0_plan"]), tt(mb["c0_plan"]))
    goal = torch.stack([F.elu(raw[..., 0]) + 0.75, torch.tanh(raw[..., 1]), torch.tanh(raw[..., 2])], -1)
    logits, _ = policy_core(Pc, ctrl_net, feat, goal, pa, masks, tt(mb["h0"]), tt(mb["c0"]))
    lp = F.log_softmax(logits, -1)
    lpa = lp.gather(2, tt(mb["action"], torch.int64)[..., None])[..., 0]
    adv = tt(mb["adv"])
    ratio = torch.exp(lpa - tt(mb["logp_old"]))
    surr = torch.min(ratio * adv, torch.clamp(ratio, 1 - ppo.clip, 1 + ppo.clip) * adv)
    ent = -(lp.exp() * lp).sum(-1)
    L = (-(w * surr).sum() + ppo.value_coef * (w * 0.5 * (values - tt(mb["ret"])) ** 2).sum()
         - ppo.entropy_coef * (w * ent).sum())
    L.backward()
    return L.item(), flat_p.grad.numpy().copy(), goal.detach().numpy()
