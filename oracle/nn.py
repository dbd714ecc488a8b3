"""Layer primitives in float64, NCHW, forward and hand-written backward.

Every function is the plain definition of the operation written out; the
only library primitives used are numpy's array slicing and tensordot
(a matrix product).

Pins (tests/test_oracle_nn.py): each forward against torch CPU float64
library routines (conv2d, group_norm, max_pool2d, avg_pool2d, the LSTM cell
equations of torch.nn.LSTMCell, log_softmax); each backward against central
finite differences and torch autograd; round_bf16 against torch's float32 to
bfloat16 conversion and against brute force over the representable values.
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

GN_EPS = 1e-5


# ------------------------------------------------------------ quantisation
def round_bf16(x):
    """Nearest bfloat16 value of each element (8 significant bits, ties to
    even), returned as float64.  Rounds the float64 value directly (no
    float32 step).  bfloat16 shares float32's exponent range; the values
    quantised here are far from its limits."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)                    # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)   # np.round: half to even


# ---------------------------------------------------------------- convolution
def _im2col(xp, KH, KW, s, Ho, Wo):
    """[B,C,Hp,Wp] -> [B,C,Ho,Wo,KH,KW] view of the receptive fields."""
    v = sliding_window_view(xp, (KH, KW), axis=(2, 3))
    return v[:, :, 0:s * (Ho - 1) + 1:s, 0:s * (Wo - 1) + 1:s]


def conv_out(H, K, s, p):
    return (H + 2 * p - K) // s + 1


def conv2d(x, w, s, p):
    """y[b,o,i,j] = sum_{c,kh,kw} xpad[b,c,s*i+kh,s*j+kw] * w[o,c,kh,kw] (no bias)."""
    B, C, H, W = x.shape
    O, C2, KH, KW = w.shape
    assert C == C2
    Ho, Wo = conv_out(H, KH, s, p), conv_out(W, KW, s, p)
    xp = np.pad(x, ((0, 0), (0, 0), (p, p), (p, p)))
    cols = _im2col(xp, KH, KW, s, Ho, Wo)
    y = np.tensordot(cols, w, axes=([1, 4, 5], [1, 2, 3]))  # [B,Ho,Wo,O]
    return np.ascontiguousarray(y.transpose(0, 3, 1, 2))


def conv2d_backward(x, w, s, p, dy, need_dx=True):
    """Gradients of conv2d with respect to its input and weight."""
    B, C, H, W = x.shape
    O, _, KH, KW = w.shape
    Ho, Wo = dy.shape[2], dy.shape[3]
    xp = np.pad(x, ((0, 0), (0, 0), (p, p), (p, p)))
    cols = _im2col(xp, KH, KW, s, Ho, Wo)
    dw = np.tensordot(dy, cols, axes=([0, 2, 3], [0, 2, 3]))  # [O,C,KH,KW]
    dx = None
    if need_dx:
        dxp = np.zeros_like(xp)
        for kh in range(KH):
            for kw in range(KW):
                contrib = np.tensordot(dy, w[:, :, kh, kw], axes=([1], [0]))  # [B,Ho,Wo,C]
                dxp[:, :, kh:kh + s * (Ho - 1) + 1:s, kw:kw + s * (Wo - 1) + 1:s] += \
                    contrib.transpose(0, 3, 1, 2)
        dx = dxp[:, :, p:p + H, p:p + W].copy()
    return dx, dw


def conv2d_grouped(x, w, s, p, groups):
    """Grouped convolution (the aggregated transform of ResNeXt): input and
    output channels are split into `groups` equal consecutive slices, and
    output slice g is the convolution of input slice g with its own filters
    w[g*O/G : (g+1)*O/G], each of which reads only C/G input channels."""
    if groups == 1:
        return conv2d(x, w, s, p)
    C, O = x.shape[1], w.shape[0]
    cg, og = C // groups, O // groups
    assert C == cg * groups and O == og * groups and w.shape[1] == cg
    return np.concatenate([conv2d(x[:, g * cg:(g + 1) * cg], w[g * og:(g + 1) * og], s, p)
                           for g in range(groups)], axis=1)


def conv2d_grouped_backward(x, w, s, p, dy, groups, need_dx=True):
    """Gradients of conv2d_grouped: each slice's own convolution gradient."""
    if groups == 1:
        return conv2d_backward(x, w, s, p, dy, need_dx)
    C, O = x.shape[1], w.shape[0]
    cg, og = C // groups, O // groups
    dxs, dws = [], []
    for g in range(groups):
        dx, dw = conv2d_backward(x[:, g * cg:(g + 1) * cg], w[g * og:(g + 1) * og], s, p,
                                 dy[:, g * og:(g + 1) * og], need_dx)
        dxs.append(dx)
        dws.append(dw)
    return (np.concatenate(dxs, axis=1) if need_dx else None), np.concatenate(dws, axis=0)


# ------------------------------------------------------------------ GroupNorm
def group_norm(x, gamma, beta, G, eps=GN_EPS):
    """Normalise each (sample, group) over its C/G channels and all pixels
    with the biased variance, then scale and shift per channel."""
    B, C, H, W = x.shape
    xr = x.reshape(B, G, -1)
    mu = xr.mean(axis=2, keepdims=True)
    var = ((xr - mu) ** 2).mean(axis=2, keepdims=True)
    rstd = 1.0 / np.sqrt(var + eps)
    xhat = ((xr - mu) * rstd).reshape(B, C, H, W)
    y = xhat * gamma[None, :, None, None] + beta[None, :, None, None]
    return y, (xhat, rstd, G)


def group_norm_backward(cache, gamma, dy):
    xhat, rstd, G = cache
    B, C, H, W = dy.shape
    dgamma = (dy * xhat).sum(axis=(0, 2, 3))
    dbeta = dy.sum(axis=(0, 2, 3))
    dxhat = (dy * gamma[None, :, None, None]).reshape(B, G, -1)
    xh = xhat.reshape(B, G, -1)
    m1 = dxhat.mean(axis=2, keepdims=True)
    m2 = (dxhat * xh).mean(axis=2, keepdims=True)
    dx = (rstd * (dxhat - m1 - xh * m2)).reshape(B, C, H, W)
    return dx, dgamma, dbeta


# ------------------------------------------------------------ squeeze-excite
def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def se_squeeze(y):
    """Per-sample, per-channel mean over the pixels: [B,C,H,W] -> [B,C]."""
    return y.mean(axis=(2, 3))


def se_excite(y, s):
    """Each channel scaled by its gate: y[b,c,:,:] * s[b,c]."""
    return y * s[:, :, None, None]


def se_excite_backward(y, s, dout):
    """Gradients of se_excite with respect to y (the direct path) and s."""
    return dout * s[:, :, None, None], (dout * y).sum(axis=(2, 3))


def linear(x, w, b):
    """x [B,I] -> x w^T + b, w [O,I]."""
    return np.tensordot(x, w, axes=([1], [1])) + b


def linear_backward(x, w, dy):
    """Gradients of linear: (dx, dw, db)."""
    return np.tensordot(dy, w, axes=([1], [0])), np.tensordot(dy, x, axes=([0], [0])), dy.sum(axis=0)


# -------------------------------------------------------------------- pooling
def avg_pool2(x):
    """Mean of non-overlapping 2x2 blocks."""
    B, C, H, W = x.shape
    return x.reshape(B, C, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def max_pool3s2(x, winner=None):
    """3x3 window, stride 2, padding 1 (padding never wins).  Returns the
    output and, per output, the flat input index of the first maximum in
    row-major window order.  `winner` ([B,C,Ho,Wo] window index kh*3+kw)
    imposes the choice instead (a decision taken elsewhere).  The cache also
    keeps the window index of every output."""
    B, C, H, W = x.shape
    Ho, Wo = conv_out(H, 3, 2, 1), conv_out(W, 3, 2, 1)
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)), constant_values=-np.inf)
    win = _im2col(xp, 3, 3, 2, Ho, Wo).reshape(B, C, Ho, Wo, 9)
    k = win.argmax(axis=4) if winner is None else np.asarray(winner, np.int64)
    y = np.take_along_axis(win, k[..., None], axis=4)[..., 0]
    kh, kw = k // 3, k % 3
    ii = 2 * np.arange(Ho)[:, None] + kh - 1    # input row of the winner
    jj = 2 * np.arange(Wo)[None, :] + kw - 1
    return y, (ii * W + jj, x.shape, k)


def max_pool3s2_backward(cache, dy):
    idx, shape = cache[:2]
    B, C, H, W = shape
    dx = np.zeros((B * C, H * W))
    flat_idx = idx.reshape(B * C, -1)
    rows = np.repeat(np.arange(B * C), flat_idx.shape[1])
    np.add.at(dx, (rows, flat_idx.ravel()), dy.reshape(B * C, -1).ravel())
    return dx.reshape(shape)


# -------------------------------------------------------------------- dense
def linear(x, w, b):
    """y = x w^T + b."""
    return x @ w.T + b


def linear_backward(x, w, dy):
    return dy @ w, dy.T @ x, dy.sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def log_softmax(z):
    m = z.max(axis=-1, keepdims=True)
    return z - m - np.log(np.exp(z - m).sum(axis=-1, keepdims=True))


# ------------------------------------------------------------------ LSTM cell
def lstm_cell(x, h, c, w, b):
    """One LSTM step; w = [W_ih | W_hh] of shape [4H, Din+H], gate blocks
    i, f, g, o."""
    H = h.shape[1]
    zz = np.concatenate([x, h], axis=1)
    a = zz @ w.T + b
    i = sigmoid(a[:, :H])
    f = sigmoid(a[:, H:2 * H])
    g = np.tanh(a[:, 2 * H:3 * H])
    o = sigmoid(a[:, 3 * H:])
    c2 = f * c + i * g
    tc = np.tanh(c2)
    h2 = o * tc
    return h2, c2, (zz, c, i, f, g, o, tc)


def lstm_cell_backward(cache, w, dh2, dc2):
    """Returns dx, dh, dc (for the inputs h, c), dw, db."""
    zz, c, i, f, g, o, tc = cache
    Din = zz.shape[1] - c.shape[1]
    do = dh2 * tc
    dc = dc2 + dh2 * o * (1.0 - tc * tc)
    di = dc * g
    dg = dc * i
    df = dc * c
    dcp = dc * f
    da = np.concatenate([di * i * (1 - i), df * f * (1 - f), dg * (1 - g * g),
                         do * o * (1 - o)], axis=1)
    dzz = da @ w
    return dzz[:, :Din], dzz[:, Din:], dcp, da.T @ zz, da.sum(axis=0)
