"""The agent of the paper's appendix "Agent Design", in float64.

  visual encoder  2x2 average pool, then either the tiny two-conv trunk or
                  the ResNet50 or SE-ResNeXt50 bottleneck layout with every
                  width halved and every BatchNorm replaced by GroupNorm
                  (Sec. 4 "Agent"; appendix "Visual Encoder"), then a 3x3
                  compression conv to a 128 x h x w map.  SE-ResNeXt blocks
                  (Xie et al., Hu et al.): bottleneck twice the ResNet's width
                  with its 3x3 convolution in `cardinality` groups, and a
                  squeeze-excite gate (reduction r) scaling the residual
                  branch per channel before the shortcut is added
  policy          flatten, FC to the hidden size (+ReLU), concatenated with
                  the goal encoding ([d, cos(theta), sin(theta)] -> FC-32)
                  and a 32-d embedding of the previous action (index 0 is the
                  start token), a stacked LSTM, and one FC giving the softmax
                  logits and the value (appendix "Navigation Policy")
Readings where the paper is silent (each listed in the design notes):
stem 7x7/2 + GroupNorm + ReLU + 3x3/2 max pool; stride on the bottleneck's
3x3; projection shortcut (1x1/s conv + GroupNorm) on the first block of a
stage; convolutions without bias; 16 groups; compression conv followed by
GroupNorm and ReLU; ReLU after the visual FC; the episode mask m_t
multiplies h and c of every layer and selects the start token.  SE-ResNeXt
(the paper gives only its name and the halving): the ResNeXt50 32x4d block
with every width halved keeps 4-channel groups at the first stage, i.e. 16
groups of a bottleneck 2w wide; squeeze-excite reduction 16 with biased FCs,
its gate applied to the branch after the block's last GroupNorm, before the
shortcut is added; stride, shortcut and stem as in the ResNet.

Parity pins: forward against torch CPU float64 library modules, backward
against torch autograd and central finite differences (tests/test_oracle_policy.py).

Discrete decisions (each ReLU's on/off pattern, each max-pool winner) can be
imposed through a `decide` dict, so that a comparison against an
implementation in another precision takes the same decisions; without it
they are taken here in float64.  A `record` dict receives every ReLU's
pre-activation and output and the max-pool input, from which `decisions`
forms the decide dict of a free run (imposing it reproduces that run bit for
bit; tests/test_oracle_decisions.py).

Precision form (quant="bf16"): the arithmetic stays float64, but every
operand of a matrix product -- the input and weight of each convolution, of
the visual FC and of each LSTM layer ([x, m h] and [W_ih | W_hh]) -- is first
rounded to the nearest bfloat16 value, the mixed-precision reading of the
design notes (GroupNorm, residual, pooling, the LSTM cell state and
pointwise math, the goal FC, the embedding and the policy/value head stay
unrounded).  Gradients pass the rounding unchanged (straight through): the
weight gradient of a product is taken against its rounded input and the
input gradient against its rounded weight.  Pinned against an independent
torch float64 model with the same rounding and straight-through autograd.
Rounding an activation to bfloat16 is itself a decision made by floating
point (which of two neighbouring codes), so in this form each activation
operand's codes can be imposed too: decide['q:' + key] holds the codes of the
operand named key (a convolution's input by the convolution's name, 'fc',
'lstm<l>.x', 'lstm<l>.h'), and record['q:' + key] receives the value the
oracle rounded.
"""
from __future__ import annotations

import numpy as np

from . import nn


# ------------------------------------------------------- precision form
QUANT_WEIGHTS = ("fc.w",)   # plus every convolution and LSTM layer weight


def quantizer(quant):
    """Operand rounding of the precision form: identity, or bfloat16."""
    if quant is None:
        return lambda a: a
    if quant == "bf16":
        return nn.round_bf16
    raise ValueError(quant)


def quantize_params(net, P, quant):
    """The parameter dict with every matrix-product weight rounded."""
    if quant is None:
        return P
    q = quantizer(quant)
    out = dict(P)
    for k, v in P.items():
        if k.startswith("lstm") and k.endswith(".w") or k in QUANT_WEIGHTS or \
                (v.ndim == 4):            # convolutions (out, in, kh, kw)
            out[k] = q(v)
    return out


# ------------------------------------------------------------------ encoder
def prep_obs(net, obs):
    x = np.asarray(obs, dtype=np.float64)
    return nn.avg_pool2(x) if net.avgpool and net.trunk != "none" else x


def _relu(y, key, decide, record=None, outputs=True):
    """ReLU with its on/off pattern taken here (y > 0) or imposed."""
    m = (y > 0) if (decide is None or key not in decide) else np.asarray(decide[key], bool)
    a = np.where(m, y, 0.0)
    if record is not None:
        record.setdefault(key, []).append(y)
        if outputs:
            record.setdefault(key + ":out", []).append(a)
    return a, m


def _operand(x, key, q, decide, record):
    """A product operand of the precision form: x rounded by q, or the codes
    imposed as decide[key]; record[key] receives x (the value before
    rounding).  q None (exact arithmetic): x unchanged."""
    if q is None:
        return x
    if record is not None:
        record.setdefault(key, []).append(x)
    if decide is not None and key in decide:
        return np.asarray(decide[key], np.float64)
    return q(x)


def _conv_gn(P, net, name, x, s, p, relu, tape, decide=None, q=None, record=None, outputs=True, groups=1):
    xq = _operand(x, "q:" + name, q, decide, record)
    u = nn.conv2d_grouped(xq, P[name], s, p, groups)
    y, gc = nn.group_norm(u, P[name + ".gn.g"], P[name + ".gn.b"], net.gn_groups)
    m = None
    if relu:
        y, m = _relu(y, name, decide, record, outputs)
    if tape is not None:
        tape[name] = (xq, s, p, gc, m, groups)
    return y


def _conv_gn_bwd(P, name, dy, tape, grads, need_dx=True):
    x, s, p, gc, m, groups = tape[name]
    if m is not None:
        dy = dy * m
    du, dg, db = nn.group_norm_backward(gc, P[name + ".gn.g"], dy)
    dx, dw = nn.conv2d_grouped_backward(x, P[name], s, p, du, groups, need_dx)
    grads[name] = grads.get(name, 0) + dw
    grads[name + ".gn.g"] = grads.get(name + ".gn.g", 0) + dg
    grads[name + ".gn.b"] = grads.get(name + ".gn.b", 0) + db
    return dx


def _se(P, pre, y, tape, decide, record, outputs):
    """Squeeze-excite gate of an SE-ResNeXt block (Hu et al.) on its residual
    branch y: z = per-channel pixel mean, h = ReLU(se1 z), s = sigmoid(se2 h),
    y scaled by s per channel.  The two FCs stay in float64 in the precision
    form (like the goal FC and the heads); the hidden ReLU is decision
    pre + 'se'."""
    z = nn.se_squeeze(y)
    h, m = _relu(nn.linear(z, P[pre + "se1.w"], P[pre + "se1.b"]), pre + "se", decide, record, outputs)
    s = nn.sigmoid(nn.linear(h, P[pre + "se2.w"], P[pre + "se2.b"]))
    if tape is not None:
        tape[pre + "se"] = (y, z, h, m, s)
    return nn.se_excite(y, s)


def _se_bwd(P, pre, d, tape, grads):
    y, z, h, m, s = tape[pre + "se"]
    dy, ds = nn.se_excite_backward(y, s, d)
    da2 = ds * s * (1.0 - s)
    dh, dw2, db2 = nn.linear_backward(h, P[pre + "se2.w"], da2)
    da1 = dh * m
    dz, dw1, db1 = nn.linear_backward(z, P[pre + "se1.w"], da1)
    for k, v in (("se1.w", dw1), ("se1.b", db1), ("se2.w", dw2), ("se2.b", db2)):
        grads[pre + k] = grads.get(pre + k, 0) + v
    hw = y.shape[2] * y.shape[3]
    return dy + dz[:, :, None, None] / hw


def _blocks(net):
    """(prefix, stride, has_projection) of every bottleneck in order."""
    out = []
    for s in range(4):
        for j in range(net.blocks[s]):
            out.append(("s%d.b%d." % (s, j), 2 if (j == 0 and s > 0) else 1, j == 0))
    return out


def encoder_forward(P, net, x, tape=None, decide=None, quant=None, record=None, record_outputs=True):
    """x: [F, C, h, w] after the optional pooling -> features [F, flat_dim]
    in channel, row, column order.  decide: optional imposed decisions keyed
    by unit name (ReLU masks, NCHW), 'sS.bJ.out' (block output ReLU),
    'sS.bJ.se' (squeeze-excite hidden ReLU, [F, C/r]) and 'maxpool' (winner
    index).  P must already be quantize_params(.., quant).
    record: optional dict of lists receiving each ReLU's pre-activation
    (key) and output (key + ':out', unless record_outputs is False) and the
    max-pool input ('maxpool')."""
    q = None if quant is None else quantizer(quant)
    cg = lambda name, a, s, p, relu: _conv_gn(P, net, name, a, s, p, relu, tape, decide, q, record,
                                              record_outputs)
    if net.trunk == "none":            # the input already is the feature vector
        return np.asarray(x, np.float64).reshape(x.shape[0], -1)
    if net.trunk == "tiny":
        a = cg("conv1", x, 2, 1, True)
        a = cg("conv2", a, 2, 1, True)
        return a.reshape(a.shape[0], -1)
    a = cg("stem", x, 2, 3, True)
    if record is not None:
        record.setdefault("maxpool", []).append(a)
    a, mc = nn.max_pool3s2(a, None if decide is None else decide.get("maxpool"))
    if tape is not None:
        tape["maxpool"] = mc
    se = net.trunk == "seresnext"
    for pre, st, proj in _blocks(net):
        y = cg(pre + "c1", a, 1, 0, True)
        if se:
            y = _conv_gn(P, net, pre + "c2", y, st, 1, True, tape, decide, q, record, record_outputs,
                         groups=net.cardinality)
        else:
            y = cg(pre + "c2", y, st, 1, True)
        y = cg(pre + "c3", y, 1, 0, False)
        if se:
            y = _se(P, pre, y, tape, decide, record, record_outputs)
        sc = cg(pre + "ds", a, st, 0, False) if proj else a
        a, m = _relu(y + sc, pre + "out", decide, record, record_outputs)
        if tape is not None:
            tape[pre + "out"] = m
    a = cg("compress", a, 1, 1, True)
    return a.reshape(a.shape[0], -1)


def encoder_backward(P, net, tape, dfeat, grads):
    """Accumulate parameter gradients for one recorded encoder forward."""
    if net.trunk == "none":
        return
    if net.trunk == "tiny":
        c2 = net.tiny_ch[1]
        hw = net.feat_hw
        d = dfeat.reshape(-1, c2, hw, hw)
        d = _conv_gn_bwd(P, "conv2", d, tape, grads)
        _conv_gn_bwd(P, "conv1", d, tape, grads, need_dx=False)
        return
    hw = net.feat_hw
    d = dfeat.reshape(-1, net.compress_ch, hw, hw)
    d = _conv_gn_bwd(P, "compress", d, tape, grads)
    for pre, st, proj in reversed(_blocks(net)):
        d = d * tape[pre + "out"]
        dy = _se_bwd(P, pre, d, tape, grads) if net.trunk == "seresnext" else d
        dy = _conv_gn_bwd(P, pre + "c3", dy, tape, grads)
        dy = _conv_gn_bwd(P, pre + "c2", dy, tape, grads)
        dx = _conv_gn_bwd(P, pre + "c1", dy, tape, grads)
        dx = dx + (_conv_gn_bwd(P, pre + "ds", d, tape, grads) if proj else d)
        d = dx
    d = nn.max_pool3s2_backward(tape["maxpool"], d)
    _conv_gn_bwd(P, "stem", d, tape, grads, need_dx=False)


def _slice(decide, s, e):
    return None if decide is None else {k: v[s:e] for k, v in decide.items()}


def encode(P, net, obs, chunk=64, decide=None, quant=None, record=None, record_outputs=True):
    """Features of many frames, processed in chunks of frames to bound the
    im2col memory (frames are independent).  record: as for encoder_forward,
    with the chunks' arrays concatenated along frames at the end."""
    F = obs.shape[0]
    if net.trunk == "none":
        return np.asarray(obs, np.float64).reshape(F, net.flat_dim)
    out = np.zeros((F, net.flat_dim))
    rec = None if record is None else {}
    for s in range(0, F, chunk):
        out[s:s + chunk] = encoder_forward(P, net, prep_obs(net, obs[s:s + chunk]),
                                           decide=_slice(decide, s, s + chunk), quant=quant, record=rec,
                                           record_outputs=record_outputs)
    if record is not None:
        for k, v in rec.items():
            record[k] = np.concatenate(v, axis=0)
    return out


def encode_backward(P, net, obs, dfeat, grads, chunk=64, decide=None, quant=None):
    """Recompute each chunk's forward with a tape, then run its backward;
    the chunk gradients are summed."""
    F = obs.shape[0]
    if net.trunk == "none":
        return
    for s in range(0, F, chunk):
        tape = {}
        encoder_forward(P, net, prep_obs(net, obs[s:s + chunk]), tape, _slice(decide, s, s + chunk), quant)
        encoder_backward(P, net, tape, dfeat[s:s + chunk], grads)


def decisions(net, record, vis_pre=None):
    """The decide dict of the run that filled `record` (encode's record of
    the encoder over frames; vis_pre [T,B,vis_hidden] the visual-FC
    pre-activations of the core): every ReLU's on/off pattern and every
    max-pool window's first maximum."""
    dec = {k: v > 0 for k, v in record.items()
           if k != "maxpool" and not k.endswith(":out") and not k.startswith("q:")}
    dec.update({k: nn.round_bf16(v) for k, v in record.items() if k.startswith("q:")})
    if "maxpool" in record:
        dec["maxpool"] = nn.max_pool3s2(record["maxpool"])[1][2]
    if vis_pre is not None:
        dec["vis"] = vis_pre > 0
    return dec


# ------------------------------------------------------------- policy core
def polar(goal):
    """[d, theta] -> [d, cos(theta), sin(theta)]."""
    d, th = goal[..., 0], goal[..., 1]
    return np.stack([d, np.cos(th), np.sin(th)], axis=-1)


def core_forward(P, net, feat, goal, prev_a, masks, h0, c0, keep=False, vis_mask=None, quant=None,
                 vis_pre=None, codes=None, qrec=None):
    """Run the policy over a sequence.

    feat [T,B,flat], goal [T,B,2], prev_a [T,B] (action taken at t-1),
    masks [T,B] (0 at an episode start), h0/c0 [L,B,H].
    vis_mask [T,B,vis_hidden] optionally imposes the visual-FC ReLU pattern;
    vis_pre (array [T,B,vis_hidden]) receives its pre-activations.
    P must already be quantize_params(.., quant).  codes: optional imposed
    operand codes 'q:fc' [T,B,flat], 'q:lstm<l>.x', 'q:lstm<l>.h' [T,B,.];
    qrec (dict) receives the values rounded, as lists over t.
    Returns logits [T,B,A], values [T,B], final (h, c), and a tape."""
    T, B = feat.shape[:2]
    L, A = net.lstm_layers, net.num_actions
    q = None if quant is None else quantizer(quant)

    def op(x, key, t):
        dec = None if codes is None or key not in codes else {key: codes[key][t]}
        return _operand(x, key, q, dec, qrec)

    h = [np.asarray(h0[l], np.float64).copy() for l in range(L)]
    c = [np.asarray(c0[l], np.float64).copy() for l in range(L)]
    logits = np.zeros((T, B, A))
    values = np.zeros((T, B))
    tape = [] if keep else None
    for t in range(T):
        m = np.asarray(masks[t], np.float64)[:, None]
        ft = op(np.asarray(feat[t], np.float64), "q:fc", t)
        pre = nn.linear(ft, P["fc.w"], P["fc.b"])
        if vis_pre is not None:
            vis_pre[t] = pre
        vis, vmask = _relu(pre, t, None if vis_mask is None else {t: vis_mask[t]})
        parts = [vis]
        g3 = None
        if net.goal_mode in ("polar", "vec3"):
            # polar: (d, theta) -> [d, cos, sin]; vec3: the 3-vector as given
            g3 = polar(np.asarray(goal[t], np.float64)) if net.goal_mode == "polar" else \
                np.asarray(goal[t], np.float64)
            parts.append(nn.linear(g3, P["goal.w"], P["goal.b"]))
        elif net.goal_mode == "raw":
            parts.append(np.asarray(goal[t], np.float64))
        idx = None
        if net.prev_act_dim:
            idx = np.where(masks[t] == 0, 0, np.asarray(prev_a[t]) + 1)
            parts.append(P["emb"][idx])
        x = np.concatenate(parts, axis=1)
        cells = []
        for l in range(L):
            h[l], c[l], cc = nn.lstm_cell(op(x, "q:lstm%d.x" % l, t), op(m * h[l], "q:lstm%d.h" % l, t), m * c[l],
                                          P["lstm%d.w" % l], P["lstm%d.b" % l])
            cells.append(cc)
            x = h[l]
        out = nn.linear(x, P["head.w"], P["head.b"])
        logits[t] = out[:, :A]
        values[t] = out[:, A]
        if keep:
            tape.append((ft, vmask, g3, idx, m, cells, x))
    return logits, values, (np.stack(h), np.stack(c)), tape


def core_backward(P, net, tape, dlogits, dvalues, grads, dgoal=None):
    """BPTT through the policy core; accumulates parameter gradients and
    returns d(feat) [T,B,flat].  dgoal (array [T,B,3], 'vec3' goal mode)
    receives the gradient with respect to the goal input."""
    T = len(tape)
    L, A = net.lstm_layers, net.num_actions
    B = dlogits.shape[1]
    H = net.hidden
    dh = [np.zeros((B, H)) for _ in range(L)]
    dc = [np.zeros((B, H)) for _ in range(L)]
    dfeat = np.zeros((T, B, net.flat_dim))
    g = {k: 0 for k in ("fc.w", "fc.b", "goal.w", "goal.b", "emb", "head.w", "head.b")}
    for l in range(L):
        g["lstm%d.w" % l] = 0
        g["lstm%d.b" % l] = 0
    emb_grad = np.zeros((net.emb_rows, net.prev_act_dim)) if net.prev_act_dim else None
    for t in reversed(range(T)):
        f_t, vmask, g3, idx, m, cells, top = tape[t]
        dout = np.concatenate([dlogits[t], dvalues[t][:, None]], axis=1)
        dtop, dwh, dbh = nn.linear_backward(top, P["head.w"], dout)
        g["head.w"] = g["head.w"] + dwh
        g["head.b"] = g["head.b"] + dbh
        dx = dtop
        for l in reversed(range(L)):
            dxl, dhp, dcp, dw, db = nn.lstm_cell_backward(
                cells[l], P["lstm%d.w" % l], dh[l] + dx, dc[l])
            g["lstm%d.w" % l] = g["lstm%d.w" % l] + dw
            g["lstm%d.b" % l] = g["lstm%d.b" % l] + db
            dh[l] = m * dhp
            dc[l] = m * dcp
            dx = dxl
        nv = net.vis_hidden
        dvis = dx[:, :nv] * vmask
        dft, dwf, dbf = nn.linear_backward(f_t, P["fc.w"], dvis)
        dfeat[t] = dft
        g["fc.w"] = g["fc.w"] + dwf
        g["fc.b"] = g["fc.b"] + dbf
        if net.goal_mode in ("polar", "vec3"):
            dgf = dx[:, nv:nv + net.goal_dim]
            dg3, dwg, dbg = nn.linear_backward(g3, P["goal.w"], dgf)
            g["goal.w"] = g["goal.w"] + dwg
            g["goal.b"] = g["goal.b"] + dbg
            if dgoal is not None:
                dgoal[t] = dg3
        if net.prev_act_dim:
            de = dx[:, nv + net.goal_dim:]
            np.add.at(emb_grad, idx, de)
    if emb_grad is not None:
        g["emb"] = emb_grad
    for k, v in g.items():
        if not isinstance(v, int):
            grads[k] = grads.get(k, 0) + v
    return dfeat


# ------------------------------------------------------------------ act step
def sample(logp, u):
    """Inverse CDF: the smallest k with sum_{j<=k} p_j > u; the last action
    if rounding leaves none."""
    cdf = np.cumsum(np.exp(logp), axis=-1)
    A = logp.shape[-1]
    hit = cdf > np.asarray(u, np.float64)[..., None]
    a = np.where(hit.any(axis=-1), hit.argmax(axis=-1), A - 1)
    return a.astype(np.int32)


def act(P, net, obs, goal, prev_a, mask, h, c, u, quant=None):
    """One batched act step for B envs: returns action, logp(action), value,
    logits, h', c'.  quant: the precision form (module header)."""
    P = quantize_params(net, P, quant)
    feat = encoder_forward(P, net, prep_obs(net, obs), quant=quant)
    logits, values, (h2, c2), _ = core_forward(
        P, net, feat[None], np.asarray(goal)[None], np.asarray(prev_a)[None],
        np.asarray(mask)[None], h, c, quant=quant)
    lp = nn.log_softmax(logits[0])
    a = sample(lp, u)
    return {"action": a, "logp": lp[np.arange(len(a)), a], "value": values[0],
            "logits": logits[0], "h": h2, "c": c2}
