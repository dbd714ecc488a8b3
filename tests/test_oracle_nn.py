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
    np.testing.assert_allclose(nn.avg_pool2(x), F.avg_pool2d(T64(x), 2).numpy(), rtol=1e-14)


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
