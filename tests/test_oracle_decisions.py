"""Pins for the oracle's imposed-decision path (ReLU patterns, max-pool
winners) and for its bfloat16 precision form.

Decisions: a run's own decisions, imposed, reproduce it bit for bit; a
single flipped decision changes exactly one output element of its layer, by
exactly the pre-activation (ReLU) or the gap to the window maximum (max
pool); with decisions held fixed the loss is smooth and its central finite
differences match the hand gradient, including at the flipped units.

Precision form: round_bf16 against torch's float32 -> bfloat16 conversion
and against brute force over every bfloat16 value; the quantised loss and
gradient against an independent torch float64 model with the same rounding
and straight-through autograd.
"""
import numpy as np
import pytest
import torch

from oracle import nn, params, policy, ppo
from synth import rollout as R
from tests import torch_ref
from tests.nets import MINI_RESNET, MINI_SERESNEXT, TINY_PLUS, wl
from tests.test_oracle_policy import random_minibatch


def _case(net, seed, T=4, B=3):
    flat = R.init_params(net, seed, random_affine=True).astype(np.float64)
    return flat, random_minibatch(net, T, B, seed=seed + 10)


def _free_run(net, flat, mb, quant=None):
    rec = {}
    s, g = ppo.loss_grad(flat, net, wl(net).ppo, mb, quant=quant, record=rec)
    return s, g, rec, policy.decisions(net, rec, rec["vis"])


# ------------------------------------------------------------ round_bf16
def test_round_bf16_matches_torch_conversion():
    g = np.random.default_rng(0)
    x = (g.standard_normal(200_000) * 10.0 ** g.uniform(-6, 6, 200_000)).astype(np.float32)
    x = np.concatenate([x, np.float32([0.0, -0.0, 1.0, -3.0])])
    want = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(nn.round_bf16(x.astype(np.float64)), want)


def test_round_bf16_brute_force_nearest_ties_even():
    # every finite bfloat16 value with exponent bits 100..150 (|v| ~ 2^-27 .. 2^24)
    bits = np.arange(1 << 16, dtype=np.uint32)
    exp = (bits >> 7) & 0xFF
    bits = bits[(exp >= 100) & (exp <= 150)]
    vals = (bits << 16).view(np.float32).astype(np.float64)
    order = np.argsort(vals)
    vals, bits = vals[order], bits[order]
    g = np.random.default_rng(1)
    x = g.choice(vals[(vals > -1e6) & (vals < 1e6)], 400)
    x = x * (1 + g.uniform(-2 ** -8, 2 ** -8, x.size))     # near and between representable values
    mids = (vals[:-1] + vals[1:]) / 2                      # exact midpoints (ties)
    x = np.concatenate([x, g.choice(mids, 100)])
    got = nn.round_bf16(x)
    for xi, gi in zip(x, got):
        d = np.abs(vals - xi)
        best = np.flatnonzero(d == d.min())
        if best.size == 2:                                 # tie: the even significand
            best = best[(bits[best] & 1) == 0]
        assert gi == vals[best[0]], (xi, gi, vals[best])


# ------------------------------------------------------------ decisions
@pytest.mark.parametrize("quant", [None, "bf16"])
@pytest.mark.parametrize("net,seed", [(TINY_PLUS, 3), (MINI_RESNET, 4), (MINI_SERESNEXT, 5)],
                         ids=["tiny+", "mini_resnet", "mini_seresnext"])
def test_imposing_own_decisions_reproduces_the_free_run(net, seed, quant):
    flat, mb = _case(net, seed)
    s0, g0, _, dec = _free_run(net, flat, mb, quant)
    s1, g1 = ppo.loss_grad(flat, net, wl(net).ppo, mb, decide=dec, quant=quant)
    assert np.array_equal(s0, s1) and np.array_equal(g0, g1)


def _fd_check(net, flat, mb, dec, g, seed, n_dir=4):
    """Central differences of the loss with the decisions held fixed."""
    f = lambda th: ppo.loss_grad(th, net, wl(net).ppo, mb, with_grad=False, decide=dec)[0][0]
    rng = np.random.default_rng(seed)
    for _ in range(n_dir):
        d = rng.standard_normal(flat.size)
        d /= np.linalg.norm(d)
        fd = (f(flat + 1e-6 * d) - f(flat - 1e-6 * d)) / 2e-6
        assert abs(fd - g @ d) <= 1e-6 * max(abs(fd), 1e-4), (fd, g @ d)


@pytest.mark.parametrize("key", ["s1.b0.c2", "s0.b0.out", "compress", "s1.b0.se"])
def test_flipped_relu_changes_one_element_by_its_preactivation(key):
    net = MINI_SERESNEXT if key.endswith(".se") else MINI_RESNET
    flat, mb = _case(net, 5)
    s0, g0, rec, dec = _free_run(net, flat, mb)
    pre = rec[key]
    j = np.unravel_index(np.argmin(np.abs(pre)), pre.shape)      # the unit nearest its kink
    flip = {k: v.copy() for k, v in dec.items()}
    flip[key][j] = ~flip[key][j]
    rec1 = {}
    s1, g1 = ppo.loss_grad(flat, net, wl(net).ppo, mb, decide=flip, record=rec1)
    np.testing.assert_array_equal(rec1[key], pre)               # upstream of the flip: unchanged
    diff = rec1[key + ":out"] - rec[key + ":out"]
    assert np.count_nonzero(diff) == 1 and diff[j] == (pre[j] if flip[key][j] else -pre[j])
    # the imposed flip is used (the loss moves), and less than a flip far from the kink
    far = np.unravel_index(np.argmax(np.abs(pre)), pre.shape)
    flip2 = {k: v.copy() for k, v in dec.items()}
    flip2[key][far] = ~flip2[key][far]
    s2, _ = ppo.loss_grad(flat, net, wl(net).ppo, mb, decide=flip2, with_grad=False)
    assert 0 < abs(s1[0] - s0[0]) < abs(s2[0] - s0[0])
    _fd_check(net, flat, mb, flip, g1, seed=7)


def test_flipped_maxpool_winner_changes_one_element_by_the_gap():
    net = MINI_RESNET
    flat, mb = _case(net, 6)
    s0, g0, rec, dec = _free_run(net, flat, mb)
    x = rec["maxpool"]
    F_, C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)), constant_values=-np.inf)
    win = np.lib.stride_tricks.sliding_window_view(xp, (3, 3), axis=(2, 3))[:, :, ::2, ::2].reshape(
        F_, C, H // 2, W // 2, 9)
    srt = np.sort(win, axis=4)
    gap = srt[..., -1] - srt[..., -2]
    gap[~np.isfinite(gap)] = np.inf
    gap[gap == 0] = np.inf                                       # ties: no second value
    j = np.unravel_index(np.argmin(gap), gap.shape)              # the closest runner-up
    second = int(np.flatnonzero(win[j] == srt[j][-2])[0])
    flip = {k: v.copy() for k, v in dec.items()}
    flip["maxpool"][j] = second
    rec1 = {}
    _, g1 = ppo.loss_grad(flat, net, wl(net).ppo, mb, decide=flip, record=rec1)
    np.testing.assert_array_equal(rec1["maxpool"], x)
    # the first unit after the pool sees the changed output: compare the pooled maps directly
    y0 = nn.max_pool3s2(x, dec["maxpool"])[0]
    y1 = nn.max_pool3s2(x, flip["maxpool"])[0]
    diff = y1 - y0
    assert np.count_nonzero(diff) == 1 and diff[j] == -gap[j]
    _fd_check(net, flat, mb, flip, g1, seed=8)


def test_flipped_visual_fc_relu():
    net = TINY_PLUS
    flat, mb = _case(net, 9)
    s0, g0, rec, dec = _free_run(net, flat, mb)
    vis = rec["vis"]
    valid = np.arange(vis.shape[0])[:, None] < mb["lens"][None, :]
    score = np.where(valid[..., None], np.abs(vis), np.inf)
    j = np.unravel_index(np.argmin(score), score.shape)
    flip = {k: v.copy() for k, v in dec.items()}
    flip["vis"][j] = ~flip["vis"][j]
    _, g1 = ppo.loss_grad(flat, net, wl(net).ppo, mb, decide=flip)
    assert not np.array_equal(g1, g0)
    _fd_check(net, flat, mb, flip, g1, seed=10)


# ------------------------------------------------------- precision form
@pytest.mark.parametrize("net,seed", [(TINY_PLUS, 11), (MINI_RESNET, 12), (MINI_SERESNEXT, 13)],
                         ids=["tiny+", "mini_resnet", "mini_seresnext"])
def test_bf16_form_matches_torch_with_straight_through_rounding(net, seed):
    flat, mb = _case(net, seed)
    s, g = ppo.loss_grad(flat, net, wl(net).ppo, mb, quant="bf16")
    L_t, g_t, _, _ = torch_ref.ppo_loss(net, wl(net).ppo, flat, mb, quant="bf16")
    assert abs(s[0] - L_t) <= 1e-11 * max(1.0, abs(L_t))
    assert np.linalg.norm(g - g_t) / np.linalg.norm(g_t) < 1e-10
    # the rounding is really applied: the form differs from the exact loss at bfloat16 scale
    s_exact, _ = ppo.loss_grad(flat, net, wl(net).ppo, mb, with_grad=False)
    assert 1e-6 < abs(s[0] - s_exact[0]) / abs(s_exact[0]) < 1e-1


def test_bf16_form_act_matches_torch():
    net = TINY_PLUS
    flat = R.init_params(net, 13, random_affine=True).astype(np.float64)
    mb = random_minibatch(net, 1, 4, seed=14, ragged=False)
    out = policy.act(params.unpack(net, flat), net, mb["obs"][0], mb["goal"][0], mb["prev_action"][0],
                     mb["mask"][0], mb["h0"], mb["c0"], np.full(4, 0.5), quant="bf16")
    _, tP = torch_ref.unpack(net, flat, requires_grad=False)
    t = lambda a, dt=torch.float64: torch.tensor(np.asarray(a), dtype=dt)
    lg, vals = torch_ref.policy_seq(tP, net, t(mb["obs"]), t(mb["goal"]), t(mb["prev_action"], torch.int64),
                                    t(mb["mask"]), t(mb["h0"]), t(mb["c0"]), quant="bf16")
    np.testing.assert_allclose(out["logits"], lg[0].numpy(), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(out["value"], vals[0].numpy(), rtol=1e-11, atol=1e-13)


# ------------------------------------------- the GPU tests' decision check
def test_decision_validator_accepts_near_kink_flips_only():
    """validate_decisions (used by the GPU parity tests on the decisions read
    back from the library): no flips for a run's own decisions, a flip at the
    kink passes and is counted, a flip far from it is rejected."""
    from tests.gpu_util import validate_decisions
    net = MINI_RESNET
    flat, mb = _case(net, 15)
    _, _, rec, dec = _free_run(net, flat, mb)
    fl = validate_decisions(dec, rec, mb["lens"], 1e-3)
    assert sum(f for _, f in fl.values()) == 0
    key = "s2.b0.c1"
    pre = rec[key]
    near = np.unravel_index(np.argmin(np.abs(pre)), pre.shape)
    far = np.unravel_index(np.argmax(np.abs(pre)), pre.shape)
    for j, ok in ((near, True), (far, False)):
        d = {k: v.copy() for k, v in dec.items()}
        d[key][j] = ~d[key][j]
        r = {}
        ppo.loss_grad(flat, net, wl(net).ppo, mb, decide=d, record=r, with_grad=False)
        if ok:
            assert validate_decisions(d, r, mb["lens"], 1e-3)[key][1] == 1
        else:
            with pytest.raises(AssertionError):
                validate_decisions(d, r, mb["lens"], 1e-3)
    # max pool: a winner that is not the window maximum, by a wide margin
    d = {k: v.copy() for k, v in dec.items()}
    x = rec["maxpool"]
    j = np.unravel_index(np.argmax(x[:, :, 2:-2:2, 2:-2:2]), x[:, :, 2:-2:2, 2:-2:2].shape)
    jo = (j[0], j[1], j[2] + 1, j[3] + 1)        # the window centred on that (interior) pixel
    d["maxpool"][jo] = 0 if dec["maxpool"][jo] != 0 else 8
    r = {}
    ppo.loss_grad(flat, net, wl(net).ppo, mb, decide=d, record=r, with_grad=False)
    with pytest.raises(AssertionError):
        validate_decisions(d, r, mb["lens"], 1e-3)


def test_imposed_operand_code_changes_one_operand_by_one_step():
    """In the bfloat16 form, replacing one imposed operand code of a
    convolution by its neighbour changes that convolution's output, seen as
    the next convolution's input value, in that frame only (the next
    operand is imposed too, so nothing else moves); the validator accepts the
    replacement where the value sits at a rounding midpoint and rejects it
    elsewhere."""
    from tests.gpu_util import validate_decisions
    net = MINI_RESNET
    flat, mb = _case(net, 17)
    s0, _, rec, dec = _free_run(net, flat, mb, quant="bf16")
    key, nxt = "q:s1.b0.c2", "q:s1.b0.c3"
    x = rec[key]
    code = nn.round_bf16(x)
    step = np.abs(nn.round_bf16(x * (1 + 2 ** -7)) - code)          # one bfloat16 step at each x
    mid_dist = np.abs(np.abs(x - code) - step / 2)                  # distance to the nearer midpoint
    for j, ok in ((np.unravel_index(np.argmin(mid_dist + (step == 0)), x.shape), True),
                  (np.unravel_index(np.argmax(np.abs(x)), x.shape), False)):
        d = {k: v.copy() for k, v in dec.items()}
        d[key][j] = code[j] + np.sign(x[j] - code[j] if x[j] != code[j] else 1.0) * step[j]
        r = {}
        ppo.loss_grad(flat, net, wl(net).ppo, mb, decide=d, quant="bf16", record=r, with_grad=False)
        np.testing.assert_array_equal(r[key], x)                     # the operand's own value: unchanged
        moved = np.any(r[nxt] != rec[nxt], axis=(1, 2, 3))
        assert moved[j[0]] and moved.sum() == 1                      # its consumer, in that frame only
        if ok:
            assert validate_decisions(d, r, mb["lens"], 1e-3, qtol=1e-4)[key][1] == 1
        else:
            with pytest.raises(AssertionError):
                validate_decisions(d, r, mb["lens"], 1e-3, qtol=1e-4)
