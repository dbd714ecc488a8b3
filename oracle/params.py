"""The oracle's own reader and writer of the flat parameter vector.

Order of tensors (one contiguous float vector): encoder trunk (convolution
weights stored output-channel, kernel-row, kernel-column, input-channel,
each followed by its GroupNorm gamma and beta; a grouped convolution stores
the input channels of its output channel's group only; an SE-ResNeXt block's
two squeeze-excite FC weights and biases follow its third convolution),
visual FC weight (input
index in channel, row, column order) and bias, goal FC (polar goal only),
previous-action embedding (if present), per LSTM layer the stacked
[W_ih | W_hh] matrix with gate row blocks i, f, g, o and one bias, and the
joint head ([A policy rows; 1 value row] and bias).

Convolution weights are returned in (out, in, kh, kw) order for nn.conv2d.
"""
from __future__ import annotations

from collections import OrderedDict

import numpy as np


def _arch(net):
    """Yield (name, shape-as-stored, is_conv) in storage order."""
    if net.trunk == "none":
        pass                       # features in: no encoder tensors
    elif net.trunk == "tiny":
        c1, c2 = net.tiny_ch
        yield "conv1", (c1, 3, 3, net.in_ch), True
        yield "conv1.gn.g", (c1,), False
        yield "conv1.gn.b", (c1,), False
        yield "conv2", (c2, 3, 3, c1), True
        yield "conv2.gn.g", (c2,), False
        yield "conv2.gn.b", (c2,), False
    else:
        base = net.base_width
        yield "stem", (base, 7, 7, net.in_ch), True
        yield "stem.gn.g", (base,), False
        yield "stem.gn.b", (base,), False
        cin = base
        se = net.trunk == "seresnext"
        for s in range(4):
            w = base << s
            # bottleneck width; SE-ResNeXt: twice the ResNet's, split into groups
            m = 2 * w if se else w
            cg = m // net.cardinality if se else m
            for j in range(net.blocks[s]):
                p = "s%d.b%d." % (s, j)
                for nm, shp in (("c1", (m, 1, 1, cin)), ("c2", (m, 3, 3, cg)),
                                ("c3", (4 * w, 1, 1, m))):
                    yield p + nm, shp, True
                    yield p + nm + ".gn.g", (shp[0],), False
                    yield p + nm + ".gn.b", (shp[0],), False
                if se:
                    r = 4 * w // net.se_reduction
                    yield p + "se1.w", (r, 4 * w), False
                    yield p + "se1.b", (r,), False
                    yield p + "se2.w", (4 * w, r), False
                    yield p + "se2.b", (4 * w,), False
                if j == 0:
                    yield p + "ds", (4 * w, 1, 1, cin), True
                    yield p + "ds.gn.g", (4 * w,), False
                    yield p + "ds.gn.b", (4 * w,), False
                cin = 4 * w
        yield "compress", (net.compress_ch, 3, 3, cin), True
        yield "compress.gn.g", (net.compress_ch,), False
        yield "compress.gn.b", (net.compress_ch,), False
    flat = net.feat_ch * net.feat_hw * net.feat_hw
    yield "fc.w", (net.vis_hidden, flat), False
    yield "fc.b", (net.vis_hidden,), False
    if net.goal_mode in ("polar", "vec3"):
        yield "goal.w", (net.goal_dim, 3), False
        yield "goal.b", (net.goal_dim,), False
    if net.prev_act_dim:
        yield "emb", (net.emb_rows, net.prev_act_dim), False
    H = net.hidden
    din = net.vis_hidden + net.goal_dim + net.prev_act_dim
    for l in range(net.lstm_layers):
        yield "lstm%d.w" % l, (4 * H, (din if l == 0 else H) + H), False
        yield "lstm%d.b" % l, (4 * H,), False
    yield "head.w", (net.num_actions + 1, H), False
    yield "head.b", (net.num_actions + 1,), False


def offsets(net):
    """name -> (offset, stored shape)."""
    out, off = OrderedDict(), 0
    for name, shp, _ in _arch(net):
        out[name] = (off, shp)
        off += int(np.prod(shp))
    return out


def count(net):
    return sum(int(np.prod(s)) for _, s, _ in _arch(net))


def unpack(net, flat):
    """Flat vector -> dict of float64 arrays (convolutions as O,I,KH,KW)."""
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.shape == (count(net),)
    P, off = {}, 0
    for name, shp, is_conv in _arch(net):
        n = int(np.prod(shp))
        a = flat[off:off + n].reshape(shp)
        P[name] = a.transpose(0, 3, 1, 2).copy() if is_conv else a.copy()
        off += n
    return P


def pack(net, D):
    """Dict in the layout of unpack() -> flat float64 vector (missing = 0)."""
    parts = []
    for name, shp, is_conv in _arch(net):
        a = D.get(name)
        if a is None:
            parts.append(np.zeros(int(np.prod(shp))))
        else:
            a = np.asarray(a, dtype=np.float64)
            parts.append((a.transpose(0, 2, 3, 1) if is_conv else a).ravel())
    return np.concatenate(parts)
