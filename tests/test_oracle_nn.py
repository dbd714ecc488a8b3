"""Pins for the oracle's layer primitives: torch CPU float64 library routines
for the forward, torch autograd and central finite differences for the
hand-written backward."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import nn

pytestmark = pytest.mark.filterwarnings("ignore")
R = np.random.default_rng(0)
T64 = lambda a: torch.tensor(a, dtype=torch.float64)


def _fd(f, x, d, h=1e-6):
    return (f(x + h * d) - f(x - h * d)) / (2 * h)


@pytest.mark.parametrize("C,O,H,K,s,p", [(3, 5, 9, 3, 1, 1), (4, 6, 10, 3, 2, 1),
                                         (4, 8, 16, 7, 2, 3), (6, 4, 7, 1, 2, 0), (5, 3, 6, 1, 1, 0)])
def test_conv2d_vs_torch(C, O, H, K, s, p):
    x = R.standard_normal((2, C, H, H + 1))
    w = R.standard_normal((O, C, K, K))
    y = nn.conv2d(x, w, s, p)
    xt, wt = T64(x).requires_grad_(), T64(w).requires_grad_()
    yt = F.conv2d(xt, wt, stride=s, padding=p)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    dy = R.standard_normal(y.shape)
    yt.backward(T64(dy))
    dx, dw = nn.conv2d_backward(x, w, s, p, dy)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dw, wt.grad.numpy(), rtol=1e-11, atol=1e-11)


def test_group_norm_vs_torch_and_fd():
    x = R.standard_normal((3, 8, 5, 4)) * 2 + 1
    g, b = R.uniform(0.5, 1.5, 8), R.uniform(-1, 1, 8)
    y, cache = nn.group_norm(x, g, b, 4)
    xt, gt, bt = T64(x).requires_grad_(), T64(g).requires_grad_(), T64(b).requires_grad_()
    yt = F.group_norm(xt, 4, gt, bt, eps=nn.GN_EPS)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    dy = R.standard_normal(y.shape)
    yt.backward(T64(dy))
    dx, dg, db = nn.group_norm_backward(cache, g, dy)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(dg, gt.grad.numpy(), rtol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-11)
    d = R.standard_normal(x.shape)
    fd = _fd(lambda xx: (nn.group_norm(xx, g, b, 4)[0] * dy).sum(), x, d)
    assert abs(fd - (dx * d).sum()) < 1e-6 * max(1, abs(fd))


def test_group_norm_constant_group_is_beta():
    x = np.ones((1, 4, 3, 3)) * 7.0
    y, _ = nn.group_norm(x, np.ones(4), np.arange(4.0), 2)
    np.testing.assert_allclose(y[0, :, 1, 1], np.arange(4.0), atol=1e-9)


def test_maxpool_vs_torch():
    x = R.standard_normal((2, 3, 9, 8))
    y, cache = nn.max_pool3s2(x)
    xt = T64(x).requires_grad_()
    yt = F.max_pool2d(xt, 3, 2, 1)
    np.testing.assert_array_equal(y, yt.detach().numpy())
    dy = R.standard_normal(y.shape)
    yt.backward(T64(dy))
    np.testing.assert_allclose(nn.max_pool3s2_backward(cache, dy), xt.grad.numpy(), atol=1e-13)


def test_maxpool_tie_goes_to_first_in_window():
    x = np.zeros((1, 1, 4, 4))      # all ties: the winner of output (0,0) is input (0,0)
    y, cache = nn.max_pool3s2(x)
    dx = nn.max_pool3s2_backward(cache, np.ones(y.shape))
    assert dx[0, 0, 0, 0] == 1 and dx.sum() == y.size


def test_avgpool_vs_torch():
    x = R.standard_normal((2, 4, 8, 6))
    # two summation orders of four float64 terms differ by a few ulps of the
    # largest term, so outputs near zero need an absolute floor
    np.testing.assert_allclose(nn.avg_pool2(x), F.avg_pool2d(T64(x), 2).numpy(), rtol=1e-14,
                               atol=4 * np.finfo(np.float64).eps * np.abs(x).max())


def test_lstm_cell_vs_torch():
    B, D, H = 3, 7, 5
    x, h, c = R.standard_normal((B, D)), R.standard_normal((B, H)), R.standard_normal((B, H))
    w, b = R.standard_normal((4 * H, D + H)), R.standard_normal(4 * H)
    h2, c2, cache = nn.lstm_cell(x, h, c, w, b)
    cell = torch.nn.LSTMCell(D, H).double()
    with torch.no_grad():
        cell.weight_ih.copy_(T64(w[:, :D]))
        cell.weight_hh.copy_(T64(w[:, D:]))
        cell.bias_ih.copy_(T64(b))
        cell.bias_hh.zero_()
    xt, ht, ct = T64(x).requires_grad_(), T64(h).requires_grad_(), T64(c).requires_grad_()
    h2t, c2t = cell(xt, (ht, ct))
    np.testing.assert_allclose(h2, h2t.detach().numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(c2, c2t.detach().numpy(), rtol=1e-12, atol=1e-14)
    dh2, dc2 = R.standard_normal((B, H)), R.standard_normal((B, H))
    ((h2t * T64(dh2)).sum() + (c2t * T64(dc2)).sum()).backward()
    dx, dh, dc, dw, db = nn.lstm_cell_backward(cache, w, dh2, dc2)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(dh, ht.grad.numpy(), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(dc, ct.grad.numpy(), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(dw[:, :D], cell.weight_ih.grad.numpy(), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(dw[:, D:], cell.weight_hh.grad.numpy(), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(db, cell.bias_ih.grad.numpy(), rtol=1e-11, atol=1e-13)


def test_log_softmax_vs_torch_and_normalised():
    z = R.standard_normal((5, 4)) * 30
    lp = nn.log_softmax(z)
    np.testing.assert_allclose(lp, F.log_softmax(T64(z), -1).numpy(), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(np.exp(lp).sum(-1), 1.0, rtol=1e-14)


@pytest.mark.parametrize("C,O,G,H,s", [(8, 8, 2, 9, 1), (16, 16, 4, 10, 2), (32, 32, 16, 8, 2), (6, 9, 3, 7, 1)])
def test_grouped_conv2d_vs_torch(C, O, G, H, s):
    """Grouped 3x3 convolution against torch's conv2d(groups=G), forward and
    autograd; groups=1 is the plain convolution."""
    x = R.standard_normal((2, C, H, H + 1))
    w = R.standard_normal((O, C // G, 3, 3))
    y = nn.conv2d_grouped(x, w, s, 1, G)
    xt, wt = T64(x).requires_grad_(), T64(w).requires_grad_()
    yt = F.conv2d(xt, wt, stride=s, padding=1, groups=G)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    dy = R.standard_normal(y.shape)
    yt.backward(T64(dy))
    dx, dw = nn.conv2d_grouped_backward(x, w, s, 1, dy, G)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dw, wt.grad.numpy(), rtol=1e-11, atol=1e-11)
    # an output channel reads its own group only: zeroing another group's input leaves it unchanged
    x2 = x.copy()
    x2[:, C // G:] = 0.0
    np.testing.assert_array_equal(nn.conv2d_grouped(x2, w, s, 1, G)[:, :O // G], y[:, :O // G])


def test_squeeze_excite_vs_torch_and_fd():
    """The SE gate's pieces (pixel mean, FC, ReLU, FC, sigmoid, channel scale)
    composed as the encoder does, against torch autograd; the sigmoid against
    its closed form at 0 and its symmetry."""
    B, C, r, H = 3, 8, 2, 5
    y = R.standard_normal((B, C, H, H))
    w1, b1 = R.standard_normal((r, C)), R.standard_normal(r)
    w2, b2 = R.standard_normal((C, r)), R.standard_normal(C)

    def fwd(y):
        z = nn.se_squeeze(y)
        a1 = nn.linear(z, w1, b1)
        h = np.maximum(a1, 0.0)
        s = nn.sigmoid(nn.linear(h, w2, b2))
        return nn.se_excite(y, s), (z, a1, h, s)

    out, (z, a1, h, s) = fwd(y)
    tt = [T64(a).requires_grad_() for a in (y, w1, b1, w2, b2)]
    zt = tt[0].mean(dim=(2, 3))
    st = torch.sigmoid(F.linear(F.relu(F.linear(zt, tt[1], tt[2])), tt[3], tt[4]))
    ot = tt[0] * st[:, :, None, None]
    np.testing.assert_allclose(out, ot.detach().numpy(), rtol=1e-13, atol=1e-13)
    d = R.standard_normal(out.shape)
    ot.backward(T64(d))
    dy, ds = nn.se_excite_backward(y, s, d)
    da2 = ds * s * (1 - s)
    dh, dw2, db2 = nn.linear_backward(h, w2, da2)
    da1 = dh * (a1 > 0)
    dz, dw1, db1 = nn.linear_backward(z, w1, da1)
    dy = dy + dz[:, :, None, None] / (H * H)
    for got, ref in zip((dy, dw1, db1, dw2, db2), tt):
        np.testing.assert_allclose(got, ref.grad.numpy(), rtol=1e-11, atol=1e-12)
    assert nn.sigmoid(np.array(0.0)) == 0.5
    v = R.standard_normal(7)
    np.testing.assert_allclose(nn.sigmoid(v) + nn.sigmoid(-v), 1.0, rtol=0, atol=1e-15)
