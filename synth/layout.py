"""Flat parameter vector format, as seen by the input generator.

The generator draws the initial FP32 parameter vector, so it has to know
where each tensor sits and what its fan-in is.  The format itself is an
interface (documented beside the C declarations); the oracle and the HIP
library each implement their own reader of it, and the tests check that the
three agree on every offset.

Order (tensor, shape):
  tiny trunk   : conv1 [c1][3][3][in_ch], gn1.g [c1], gn1.b [c1],
                 conv2 [c2][3][3][c1],    gn2.g [c2], gn2.b [c2]
  resnet trunk : stem [w0][7][7][in_ch], stem.gn.g/b [w0];
                 per stage s, per block j:
                   c1 [w][1][1][cin], gn1.g/b [w], c2 [w][3][3][w], gn2.g/b [w],
                   c3 [4w][1][1][w], gn3.g/b [4w],
                   (block 0 only) ds [4w][1][1][cin], ds.gn.g/b [4w];
                 compress [cc][3][3][8*w0*4], compress.gn.g/b [cc]
  seresnext    : as resnet with m = 2w: c1 [m][1][1][cin], c2 [m][3][3][m/card]
                 (grouped: output channel o reads input channels of group
                 o // (m/card)), c3 [4w][1][1][m], each with its GroupNorm, then
                 se1.w [4w/r][4w], se1.b [4w/r], se2.w [4w][4w/r], se2.b [4w],
                 then (block 0 only) ds
  visual FC    : fc.w [vis_hidden][flat_dim] (input index in C,H,W order), fc.b
  goal FC      : goal.w [goal_dim][3], goal.b [goal_dim]     (polar or 3-vector goal only)
  trunk 'none' : no encoder tensors (the visual FC reads in_ch-wide features)
  prev action  : emb [A'+1][prev_act_dim], A' = prev_actions or num_actions (if prev_act_dim > 0)
  LSTM layer l : lstm{l}.w [4H][in_l + H] (input columns, then recurrent columns;
                 gate row blocks i, f, g, o), lstm{l}.b [4H]
  heads        : head.w [A+1][H] (rows 0..A-1 policy logits, row A value), head.b [A+1]
Convolution weights are O,KH,KW,I ordered.
"""
from __future__ import annotations

from typing import List, NamedTuple, Tuple

from .configs import NetDesc


class Tensor(NamedTuple):
    name: str
    shape: Tuple[int, ...]
    kind: str        # 'conv' | 'fc' | 'bias' | 'gn_g' | 'gn_b' | 'emb'
    fan_in: int
    offset: int


def tensor_list(net: NetDesc) -> List[Tensor]:
    out: List[Tensor] = []
    off = 0

    def add(name, shape, kind, fan_in=0):
        nonlocal off
        n = 1
        for s in shape:
            n *= s
        out.append(Tensor(name, tuple(shape), kind, fan_in, off))
        off += n

    def conv(name, co, k, ci):
        add(name, (co, k, k, ci), "conv", k * k * ci)

    def gn(name, c):
        add(name + ".g", (c,), "gn_g")
        add(name + ".b", (c,), "gn_b")

    if net.trunk == "none":
        pass                       # features in: no encoder tensors
    elif net.trunk == "tiny":
        c1, c2 = net.tiny_ch
        conv("enc.conv1", c1, 3, net.in_ch)
        gn("enc.gn1", c1)
        conv("enc.conv2", c2, 3, c1)
        gn("enc.gn2", c2)
    else:
        w0 = net.base_width
        conv("enc.stem", w0, 7, net.in_ch)
        gn("enc.stem.gn", w0)
        cin = w0
        se = net.trunk == "seresnext"
        for s, nb in enumerate(net.blocks):
            w = w0 * (2 ** s)
            m = net.mid_width(s)
            for j in range(nb):
                p = f"enc.s{s}.b{j}"
                conv(p + ".c1", m, 1, cin)
                gn(p + ".gn1", m)
                conv(p + ".c2", m, 3, m // net.cardinality if se else m)
                gn(p + ".gn2", m)
                conv(p + ".c3", 4 * w, 1, m)
                gn(p + ".gn3", 4 * w)
                if se:
                    r = 4 * w // net.se_reduction
                    add(p + ".se1.w", (r, 4 * w), "fc", 4 * w)
                    add(p + ".se1.b", (r,), "bias")
                    add(p + ".se2.w", (4 * w, r), "fc", r)
                    add(p + ".se2.b", (4 * w,), "bias")
                if j == 0:
                    conv(p + ".ds", 4 * w, 1, cin)
                    gn(p + ".ds.gn", 4 * w)
                cin = 4 * w
        conv("enc.compress", net.compress_ch, 3, cin)
        gn("enc.compress.gn", net.compress_ch)
    add("fc.w", (net.vis_hidden, net.flat_dim), "fc", net.flat_dim)
    add("fc.b", (net.vis_hidden,), "bias")
    if net.goal_mode in ("polar", "vec3"):
        add("goal.w", (net.goal_dim, 3), "fc", 3)
        add("goal.b", (net.goal_dim,), "bias")
    if net.prev_act_dim > 0:
        add("emb", (net.emb_rows, net.prev_act_dim), "emb")
    H = net.hidden
    for l in range(net.lstm_layers):
        nin = net.lstm_in if l == 0 else H
        add(f"lstm{l}.w", (4 * H, nin + H), "fc", nin + H)
        add(f"lstm{l}.b", (4 * H,), "bias")
    add("head.w", (net.num_actions + 1, H), "fc", H)
    add("head.b", (net.num_actions + 1,), "bias")
    return out


def param_count(net: NetDesc) -> int:
    t = tensor_list(net)[-1]
    n = 1
    for s in t.shape:
        n *= s
    return t.offset + n
