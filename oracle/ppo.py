"""The learner side of one DD-PPO worker, in float64.

  rollout     T+1 dependent act steps (the last one only for the bootstrap
              value), Sec. 3 / Sec. 4 "Training"
  gae         generalized advantage estimation with gamma and the GAE
              parameter (called tau in Sec. 4 "Training"); an episode end
              stops both the bootstrap and the accumulation; a rollout cut
              short by preemption (Sec. 3) is bootstrapped with the value of
              its last observation
  adv_stats   population mean and variance of the advantages (reported;
              normalisation is off by default, Sec. 4 "Training")
  loss_grad   the clipped surrogate of Eq. 2 with ratio r_t of Sec. 2, plus
              a 1/2 squared-error value loss and an entropy bonus; every
              env's rollout is weighted equally (Sec. 3: 1/(|B| T_n) per
              step); hand-written gradient
  adam        Kingma & Ba's update with bias correction (the ParamUpdate
              of Eq. 3, with the all-reduce being the identity on one worker)
  update      E epochs x M minibatches of whole env sequences (Sec. 4)

Pins (tests/test_oracle_ppo.py): GAE against its closed forms at lambda=0
(TD error) and lambda=1 (discounted return minus value, Eq. 1 / Sec. 2),
episode resets, and a brute-force double sum; the surrogate against the
ratio-1 invariant and the clipping special cases; the gradient against
finite differences and torch autograd; Adam's first step against its closed
form and torch.optim.Adam.
"""
from __future__ import annotations

import numpy as np

from . import nn, params, policy

STAT_NAMES = ("loss", "pg", "vf", "ent", "clip_frac", "approx_kl", "ratio_min", "ratio_max")


# ------------------------------------------------------------------ rollout
def rollout(flat, net, inp, h0, c0, prev_a0=None, mask0=None, forced_actions=None, quant=None):
    """Collect one rollout with T+1 act steps.  inp holds obs, goal, done, u,
    lengths.  Env n is active at act step t when t <= T_n; the step t = T_n
    only provides the bootstrap value.  If forced_actions [T+1,N] is given,
    those actions (not the sampled ones) feed the previous-action input.
    quant: the precision form of policy (None: exact float64)."""
    P = params.unpack(net, flat)
    obs, goal, done, u, lens = inp["obs"], inp["goal"], inp["done"], inp["u"], inp["lengths"]
    T1, N = u.shape
    L, H = net.lstm_layers, net.hidden
    h = np.asarray(h0, np.float64).copy()
    c = np.asarray(c0, np.float64).copy()
    prev = np.zeros(N, np.int32) if prev_a0 is None else np.asarray(prev_a0, np.int32).copy()
    m = np.zeros(N) if mask0 is None else np.asarray(mask0, np.float64).copy()
    rec = {k: np.zeros((T1, N)) for k in ("logp", "value", "mask")}
    rec["action"] = np.zeros((T1, N), np.int32)
    rec["prev_action"] = np.zeros((T1, N), np.int32)
    rec["logits"] = np.zeros((T1, N, net.num_actions))
    rec["h0"], rec["c0"] = h.copy(), c.copy()
    for t in range(T1):
        act_ix = np.nonzero(t <= lens)[0]
        if t > 0:
            m = 1.0 - done[t - 1].astype(np.float64)
        o = policy.act(P, net, obs[t, act_ix], goal[t, act_ix], prev[act_ix], m[act_ix],
                       h[:, act_ix], c[:, act_ix], u[t, act_ix], quant=quant)
        rec["mask"][t] = m
        rec["prev_action"][t] = prev
        for k in ("logp", "value", "action", "logits"):
            rec[k][t, act_ix] = o[k]
        h[:, act_ix] = o["h"]
        c[:, act_ix] = o["c"]
        a_next = o["action"] if forced_actions is None else forced_actions[t, act_ix]
        prev[act_ix] = a_next
    rec["h_end"], rec["c_end"] = h, c
    return rec


# ---------------------------------------------------------------------- GAE
def gae(rew, val, done, lengths, gamma, lam):
    """rew, done [T,N]; val [T+1,N]; lengths [N].  Returns advantages and
    returns [T,N] (zero past each env's length)."""
    T, N = rew.shape
    adv = np.zeros((T, N))
    for n in range(N):
        a_next = 0.0
        for t in reversed(range(int(lengths[n]))):
            keep = 1.0 - float(done[t, n])
            delta = float(rew[t, n]) + gamma * keep * float(val[t + 1, n]) - float(val[t, n])
            a_next = delta + gamma * lam * keep * a_next
            adv[t, n] = a_next
    valid = np.arange(T)[:, None] < np.asarray(lengths)[None, :]
    ret = np.where(valid, adv + np.asarray(val[:T], np.float64), 0.0)
    return adv, ret


def adv_stats(adv, lengths):
    """Population mean and variance of the valid advantages (two passes)."""
    T = adv.shape[0]
    valid = np.arange(T)[:, None] < np.asarray(lengths)[None, :]
    x = adv[valid]
    mu = x.sum() / x.size
    var = ((x - mu) ** 2).sum() / x.size
    return mu, var


# --------------------------------------------------------------------- loss
def minibatch_inputs(net, inp, rec, adv, ret, envs):
    """Slice one minibatch (env set) out of the rollout; time-major [T_B, B]."""
    lens = np.asarray(inp["lengths"])[envs]
    TB = int(lens.max())
    return {
        "envs": envs, "lens": lens,
        "obs": inp["obs"][:TB][:, envs], "goal": inp["goal"][:TB][:, envs],
        "prev_action": rec["prev_action"][:TB][:, envs], "mask": rec["mask"][:TB][:, envs],
        "action": rec["action"][:TB][:, envs], "logp_old": rec["logp"][:TB][:, envs],
        "adv": adv[:TB][:, envs], "ret": ret[:TB][:, envs],
        "h0": rec["h0"][:, envs], "c0": rec["c0"][:, envs],
    }


def objective(logits, values, mb, ppo, adv_norm=None, with_grad=True):
    """The PPO objective of one minibatch on given policy outputs (logits
    [T_B,B,A], values [T_B,B]):
      L = -sum_n w_n sum_t min(r A, clip(r, 1-eps, 1+eps) A)
          + c_v sum_n w_n sum_t 1/2 (V - R)^2 - c_e sum_n w_n sum_t H(pi),
      w_n = 1 / (|B| T_n) (Eq. 2, Sec. 3).  Returns the statistics [8] and,
    with_grad, dL/dlogits and dL/dvalues (else None, None)."""
    lens = mb["lens"]
    TB, B = mb["action"].shape
    A_ = logits.shape[2]
    valid = np.arange(TB)[:, None] < lens[None, :]
    w = valid / (B * lens[None, :].astype(np.float64))
    lp = nn.log_softmax(logits)
    p = np.exp(lp)
    a = mb["action"]
    lpa = np.take_along_axis(lp, a[..., None], axis=2)[..., 0]
    adv = np.asarray(mb["adv"], np.float64)
    if adv_norm is not None:
        adv = (adv - adv_norm[0]) / (np.sqrt(adv_norm[1]) + 1e-5)
    ratio = np.exp(lpa - mb["logp_old"])
    s1 = ratio * adv
    s2 = np.clip(ratio, 1 - ppo.clip, 1 + ppo.clip) * adv
    surr = np.minimum(s1, s2)
    ent = -(p * lp).sum(axis=2)
    L_pg = -(w * surr).sum()
    L_v = (w * 0.5 * (values - mb["ret"]) ** 2).sum()
    L_H = (w * ent).sum()
    loss = L_pg + ppo.value_coef * L_v - ppo.entropy_coef * L_H
    clipped = np.abs(ratio - 1.0) > ppo.clip
    stats = np.array([loss, L_pg, L_v, L_H, (w * clipped).sum(),
                      (w * (mb["logp_old"] - lpa)).sum(),
                      ratio[valid].min(), ratio[valid].max()])
    if not with_grad:
        return stats, None, None
    # d/d logp(a): the unclipped branch (taken at ties) carries r*A
    dlpa = np.where(s1 <= s2, -w * adv * ratio, 0.0)
    onehot = np.eye(A_)[a]
    dlogits = dlpa[..., None] * (onehot - p)
    dlogits += ppo.entropy_coef * w[..., None] * p * (lp + ent[..., None])
    dvalues = ppo.value_coef * w * (values - mb["ret"])
    return stats, dlogits, dvalues


def loss_grad(flat, net, ppo, mb, with_grad=True, adv_norm=None, decide=None, quant=None, record=None,
              record_outputs=True):
    """PPO loss of one minibatch and (optionally) its flat gradient.

    L = -sum_n w_n sum_t min(r A, clip(r, 1-eps, 1+eps) A)
        + c_v sum_n w_n sum_t 1/2 (V - R)^2 - c_e sum_n w_n sum_t H(pi),
    w_n = 1 / (|B| T_n).  adv_norm = (mean, var) applies (A - mean)/(std + 1e-5).
    decide: optional imposed ReLU / max-pool decisions (policy.encoder_forward),
    per valid frame in time-major order, plus 'vis' [T_B, B, vis_hidden].
    quant: the precision form of policy (None: exact float64).
    record: optional dict receiving the encoder's pre-activations, outputs
    and max-pool inputs per valid frame (policy.encode) and 'vis' [T_B, B,
    vis_hidden] (visual-FC pre-activations; invalid frames 0), and in the
    bfloat16 form the values each operand rounded ('q:' keys; the core's
    time-major); record_outputs False leaves out the ReLU outputs (key +
    ':out');
    policy.decisions(net, record, record['vis']) is then this run's decide."""
    P = policy.quantize_params(net, params.unpack(net, flat), quant)
    lens = mb["lens"]
    TB, B = mb["action"].shape
    A_ = net.num_actions
    valid = np.arange(TB)[:, None] < lens[None, :]
    w = valid / (B * lens[None, :].astype(np.float64))
    # encoder over valid frames only
    tt, jj = np.nonzero(valid)
    feat = np.zeros((TB, B, net.flat_dim))
    core_keys = lambda k: k == "vis" or k.startswith("q:fc") or k.startswith("q:lstm")
    enc_decide = None if decide is None else {k: v for k, v in decide.items() if not core_keys(k)}
    codes = None if decide is None else {k: v for k, v in decide.items() if k.startswith("q:") and core_keys(k)}
    enc_rec = None if record is None else {}
    feat[tt, jj] = policy.encode(P, net, mb["obs"][tt, jj], decide=enc_decide, quant=quant, record=enc_rec,
                                 record_outputs=record_outputs)
    vis_pre = None if record is None else np.zeros((TB, B, net.vis_hidden))
    qrec = None if record is None else {}
    logits, values, _, tape = policy.core_forward(
        P, net, feat, mb["goal"], mb["prev_action"], mb["mask"], mb["h0"], mb["c0"], keep=with_grad,
        vis_mask=None if decide is None else decide.get("vis"), quant=quant, vis_pre=vis_pre, codes=codes,
        qrec=qrec)
    if record is not None:
        record.update(enc_rec)
        record["vis"] = np.where(valid[..., None], vis_pre, 0.0)
        for k, v in qrec.items():     # time-major [T_B, B, .]; invalid frames 0
            record[k] = np.where(valid[..., None], np.stack(v), 0.0)
    stats, dlogits, dvalues = objective(logits, values, mb, ppo, adv_norm, with_grad)
    if not with_grad:
        return stats, None
    grads = {}
    dfeat = policy.core_backward(P, net, tape, dlogits, dvalues, grads)
    policy.encode_backward(P, net, mb["obs"][tt, jj], dfeat[tt, jj], grads, decide=enc_decide, quant=quant)
    return stats, params.pack(net, grads)


# --------------------------------------------------------------------- Adam
def adam(theta, g, m, v, k, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Step k (1-based) of Adam with bias correction."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** k)
    vh = v / (1 - b2 ** k)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------- update
def update(flat, net, ppo, inp, rec, parts):
    """GAE, then for every epoch and minibatch a loss gradient and an Adam
    step (the all-reduce of Eq. 4 is the identity on one worker)."""
    adv, ret = gae(inp["reward"], rec["value"], inp["done"], inp["lengths"], ppo.gamma, ppo.lam)
    mu, var = adv_stats(adv, inp["lengths"])
    theta = np.asarray(flat, np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    k = 0
    log = []
    for ep in parts:
        for envs in ep:
            mb = minibatch_inputs(net, inp, rec, adv, ret, np.asarray(envs))
            stats, g = loss_grad(theta, net, ppo, mb,
                                 adv_norm=(mu, var) if ppo.norm_adv else None)
            k += 1
            theta, m, v = adam(theta, g, m, v, k, ppo.lr, ppo.beta1, ppo.beta2, ppo.eps)
            log.append((stats, g))
    return {"theta": theta, "m": m, "v": v, "k": k, "adv": adv, "ret": ret,
            "adv_mean": mu, "adv_var": var, "log": log}
