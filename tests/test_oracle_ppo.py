"""Pins for GAE, advantage statistics, the clipped surrogate and Adam."""
import math

import numpy as np
import pytest
import torch
from hypothesis import given, settings, strategies as st

from oracle import nn, params, policy, ppo
from synth import rollout as R
from synth.configs import PPOCfg
from tests import torch_ref
from tests.nets import TINY_NET, TINY_PLUS, wl
from tests.test_oracle_policy import random_minibatch


def _episode(T, N, seed, p_done=0.2):
    g = np.random.default_rng(seed)
    return (g.standard_normal((T, N)), g.standard_normal((T + 1, N)),
            (g.random((T, N)) < p_done).astype(np.uint8))


def gae_brute(rew, val, done, lens, gamma, lam):
    """A_t = sum_l (gamma lam)^l prod_{j<l} (1 - d_{t+j}) delta_{t+l}  (O(T^2))."""
    T, N = rew.shape
    A = np.zeros((T, N))
    for n in range(N):
        Tn = int(lens[n])
        delta = [rew[t, n] + gamma * (1 - done[t, n]) * val[t + 1, n] - val[t, n] for t in range(Tn)]
        for t in range(Tn):
            s, keep = 0.0, 1.0
            for l in range(Tn - t):
                s += (gamma * lam) ** l * keep * delta[t + l]
                keep *= 1 - done[t + l, n]
            A[t, n] = s
    return A


def test_gae_lambda0_is_td_error():
    rew, val, done = _episode(9, 3, 0)
    A, ret = ppo.gae(rew, val, done, [9, 9, 9], 0.99, 0.0)
    td = rew + 0.99 * (1 - done) * val[1:] - val[:-1]
    np.testing.assert_allclose(A, td, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(ret, A + val[:-1], rtol=1e-14)


def test_gae_lambda1_no_done_is_discounted_return_minus_value():
    """Eq. 1 / Sec. 2: with no episode end and a zero bootstrap value,
    A_t = sum_{i>=t} gamma^(i-t) r_i - V_t."""
    T, g = 12, 0.99
    rew, val, _ = _episode(T, 2, 1)
    val[T] = 0.0
    A, _ = ppo.gae(rew, val, np.zeros((T, 2), np.uint8), [T, T], g, 1.0)
    for t in range(T):
        Rt = sum(g ** (i - t) * rew[i] for i in range(t, T))
        np.testing.assert_allclose(A[t], Rt - val[t], rtol=1e-12, atol=1e-12)


def test_gae_lambda1_with_done_truncates_at_episode_end():
    T, g = 10, 0.9
    rew, val, _ = _episode(T, 1, 2)
    done = np.zeros((T, 1), np.uint8)
    done[4] = 1
    A, _ = ppo.gae(rew, val, done, [T], g, 1.0)
    for t in range(T):
        e = 5 if t <= 4 else T
        boot = 0.0 if e == 5 else g ** (e - t) * val[e, 0]
        Rt = sum(g ** (i - t) * rew[i, 0] for i in range(t, e)) + boot
        assert abs(A[t, 0] - (Rt - val[t, 0])) < 1e-12


def test_gae_done_resets_isolate_episodes():
    rew, val, done = _episode(8, 1, 3, p_done=0.0)
    done[3] = 1
    A1, _ = ppo.gae(rew, val, done, [8], 0.99, 0.95)
    rew2, val2 = rew.copy(), val.copy()
    rew2[4:] += 5.0
    val2[4:] -= 3.0
    A2, _ = ppo.gae(rew2, val2, done, [8], 0.99, 0.95)
    np.testing.assert_array_equal(A1[:4], A2[:4])


def test_gae_truncated_rollout_bootstraps_from_last_value():
    """A rollout cut at T_n (preemption, Sec. 3) bootstraps with V[T_n]."""
    rew, val, done = _episode(6, 1, 4, p_done=0.0)
    A, _ = ppo.gae(rew, val, done, [3], 0.99, 0.95)
    assert abs(A[2, 0] - (rew[2, 0] + 0.99 * val[3, 0] - val[2, 0])) < 1e-14
    assert np.all(A[3:] == 0)


@settings(max_examples=60, deadline=None)
@given(T=st.integers(1, 12), N=st.integers(1, 4), gamma=st.floats(0.5, 1.0),
       lam=st.floats(0.0, 1.0), seed=st.integers(0, 10_000), ragged=st.booleans())
def test_gae_matches_brute_force(T, N, gamma, lam, seed, ragged):
    rew, val, done = _episode(T, N, seed)
    lens = np.random.default_rng(seed).integers(1, T + 1, N) if ragged else np.full(N, T)
    A, _ = ppo.gae(rew, val, done, lens, gamma, lam)
    np.testing.assert_allclose(A, gae_brute(rew, val, done, lens, gamma, lam), rtol=1e-11, atol=1e-11)


def test_adv_stats_vs_fsum_and_constant():
    g = np.random.default_rng(5)
    A = g.standard_normal((20, 4)) * 3 + 2
    lens = np.array([20, 7, 13, 1])
    mu, var = ppo.adv_stats(A, lens)
    vals = [A[t, n] for n in range(4) for t in range(lens[n])]
    m = math.fsum(vals) / len(vals)
    assert abs(mu - m) < 1e-14
    assert abs(var - math.fsum((x - m) ** 2 for x in vals) / len(vals)) < 1e-13
    assert ppo.adv_stats(np.full((5, 2), 0.7), [5, 5])[1] < 1e-30


# ----------------------------------------------------------- surrogate
def _current_logp(net, flat, mb):
    P = params.unpack(net, flat)
    TB, B = mb["action"].shape
    feat = policy.encode(P, net, mb["obs"].reshape(TB * B, *mb["obs"].shape[2:])).reshape(TB, B, -1)
    lg, vals, _, _ = policy.core_forward(P, net, feat, mb["goal"], mb["prev_action"], mb["mask"],
                                         mb["h0"], mb["c0"])
    lp = nn.log_softmax(lg)
    return np.take_along_axis(lp, mb["action"][..., None], 2)[..., 0], lp


def test_ratio_one_gives_vanilla_policy_gradient():
    """Eq. 2 at r = 1: min(rA, clip(r)A) = A, so L_pg = -sum w A and its
    gradient is the plain policy gradient -sum w A grad log pi(a)."""
    net = TINY_PLUS
    cfg = PPOCfg(value_coef=0.0, entropy_coef=0.0)
    flat = R.init_params(net, 11, random_affine=True).astype(np.float64)
    mb = random_minibatch(net, 4, 3, seed=12, ragged=False)
    mb["logp_old"], _ = _current_logp(net, flat, mb)
    stats, g = ppo.loss_grad(flat, net, cfg, mb)
    w = 1.0 / (3 * 4)
    assert abs(stats[1] - (-w * mb["adv"].sum())) < 1e-13
    assert abs(stats[6] - 1) < 1e-13 and abs(stats[7] - 1) < 1e-13
    # vanilla policy gradient via torch autograd
    flat_t, P = torch_ref.unpack(net, flat)
    t = lambda a, dt=torch.float64: torch.tensor(np.asarray(a), dtype=dt)
    lg, _ = torch_ref.policy_seq(P, net, t(mb["obs"]), t(mb["goal"]), t(mb["prev_action"], torch.int64),
                                 t(mb["mask"]), t(mb["h0"]), t(mb["c0"]))
    lpa = torch.log_softmax(lg, -1).gather(2, t(mb["action"], torch.int64)[..., None])[..., 0]
    (-(w * t(mb["adv"]) * lpa).sum()).backward()
    np.testing.assert_allclose(g, flat_t.grad.numpy(), rtol=1e-9, atol=1e-14)


def test_clipped_region_has_zero_policy_gradient():
    """A > 0 with r > 1+eps, and A < 0 with r < 1-eps: the clipped term is
    the minimum and carries no gradient."""
    net = TINY_PLUS
    cfg = PPOCfg(value_coef=0.0, entropy_coef=0.0)
    flat = R.init_params(net, 13, random_affine=True).astype(np.float64)
    mb = random_minibatch(net, 3, 2, seed=14, ragged=False)
    lpa, _ = _current_logp(net, flat, mb)
    mb["logp_old"] = np.where(mb["adv"] > 0, lpa - 0.5, lpa + 0.5)
    stats, g = ppo.loss_grad(flat, net, cfg, mb)
    assert np.all(g == 0.0)
    assert stats[4] == pytest.approx(1.0)
    # the loss is the clipped value
    w = 1.0 / 6
    exp = -(w * np.where(mb["adv"] > 0, 1.2, 0.8) * mb["adv"]).sum()
    assert abs(stats[1] - exp) < 1e-13


def test_uniform_policy_entropy_is_log_A_with_zero_gradient():
    net = TINY_NET
    flat = R.init_params(net, 15).astype(np.float64)
    P = params.unpack(net, flat)
    hw = params.offsets(net)["head.w"][0]
    flat[hw:hw + 4 * net.hidden] = 0.0              # logits rows of the head -> 0
    flat[params.offsets(net)["head.b"][0]:][:4] = 0.0
    cfg = PPOCfg(value_coef=0.0, entropy_coef=1.0)
    mb = random_minibatch(net, 3, 2, seed=16, ragged=False)
    mb["adv"][:] = 0.0
    stats, g = ppo.loss_grad(flat, net, cfg, mb)
    assert abs(stats[3] - math.log(4)) < 1e-14
    assert np.abs(g).max() < 1e-15


# ------------------------------------------------------------------ Adam
def test_adam_first_step_closed_form():
    g = np.random.default_rng(6).standard_normal(100)
    th0 = np.random.default_rng(7).standard_normal(100)
    th1, m, v = ppo.adam(th0, g, np.zeros(100), np.zeros(100), 1, 2.5e-4)
    np.testing.assert_allclose(th1, th0 - 2.5e-4 * g / (np.abs(g) + 1e-8), rtol=1e-15, atol=1e-18)


def test_adam_vs_torch_optim():
    rng = np.random.default_rng(8)
    th = rng.standard_normal(50)
    p = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=2.5e-4, betas=(0.9, 0.999), eps=1e-8)
    m = v = np.zeros(50)
    for k in range(1, 5):
        g = rng.standard_normal(50)
        th, m, v = ppo.adam(th, g, m, v, k, 2.5e-4)
        p.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


# --------------------------------------------------------- whole update
def test_rollout_then_first_minibatch_ratio_is_one():
    """The learner re-evaluates the rollout's own actions with the rollout's
    parameters at the first minibatch, so every ratio is 1."""
    w = wl(TINY_PLUS, T=6, N=4, ragged=True, epochs=1, minibatches=2)
    flat = R.init_params(w.net, 17, random_affine=True)
    inp = R.gen_rollout(w.with_(net=w.net), 17)
    inp["obs"] = R.gen_obs(w.net, w.T + 1, w.N, 17, 0, False)
    inp["lengths"] = np.array([6, 3, 5, 2], np.int32)
    h0, c0 = R.gen_state(w.net, w.N, 17, zero=False)
    rec = ppo.rollout(flat, w.net, inp, h0, c0)
    out = ppo.update(flat, w.net, w.ppo, inp, rec, [[np.array([0, 2]), np.array([1, 3])]])
    s = out["log"][0][0]
    assert abs(s[6] - 1) < 1e-12 and abs(s[7] - 1) < 1e-12
    assert out["k"] == 2
