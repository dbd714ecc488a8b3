"""Parity of every C-ABI call against the FP64 oracle on the same seeded
inputs (GPU).  Tolerances: float32 path 1e-4 relative, bfloat16 path 2e-2
relative (per output tensor, relative L2)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import params as OP, policy, ppo
from synth import rollout as R
from synth.configs import C0, C1, PPOCfg
from tests.gpu_util import DEV, oracle_minibatch, per_tensor_errors, random_record, rel_err, to_device
from tests.nets import MINI_RESNET, RESNET_64, RESNET_SMALLCORE, TINY_BIGCORE, TINY_CORE1024, TINY_NET, TINY_PLUS

pytestmark = pytest.mark.gpu
TOL = {"f32": 1e-4, "bf16": 2e-2}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ---------------------------------------------------------------- GAE
@pytest.mark.parametrize("T,N,ragged,seed", [(16, 2, False, 0), (128, 4, False, 1), (128, 64, True, 2),
                                             (1, 3, False, 3), (200, 5, True, 4), (64, 1, False, 5)])
def test_gae_parity(P, T, N, ragged, seed):
    say(f"gae T={T} N={N} ragged={ragged}")
    g = np.random.default_rng(seed)
    rew = (-0.01 + 0.05 * g.standard_normal((T, N))).astype(np.float32)
    done = (g.random((T, N)) < 0.05).astype(np.uint8)
    rew += 2.5 * done
    val = g.standard_normal((T + 1, N)).astype(np.float32)
    lens = g.integers(max(1, T // 4), T + 1, N).astype(np.int32) if ragged else np.full(N, T, np.int32)
    stats = torch.zeros(2, dtype=torch.float64, device=DEV)
    adv, ret = P.gae(torch.tensor(rew, device=DEV), torch.tensor(val, device=DEV),
                     torch.tensor(done, device=DEV), torch.tensor(lens, device=DEV) if ragged else None,
                     0.99, 0.95, stats=stats)
    A, Rt = ppo.gae(rew, val, done, lens, 0.99, 0.95)
    torch.cuda.synchronize()
    assert rel_err(adv.cpu().numpy(), A) < 1e-5
    assert rel_err(ret.cpu().numpy(), Rt) < 1e-5
    mu, var = ppo.adv_stats(A, lens)
    s = stats.cpu().numpy()
    assert abs(s[0] - mu) < 1e-6 * max(1, abs(mu)) and abs(s[1] - var) < 1e-5 * var


def test_gae_closed_form_lambda0(P):
    g = np.random.default_rng(9)
    T, N = 33, 3
    rew = g.standard_normal((T, N)).astype(np.float32)
    val = g.standard_normal((T + 1, N)).astype(np.float32)
    done = (g.random((T, N)) < 0.2).astype(np.uint8)
    adv, _ = P.gae(torch.tensor(rew, device=DEV), torch.tensor(val, device=DEV),
                   torch.tensor(done, device=DEV), None, 0.9, 0.0)
    td = rew.astype(np.float64) + 0.9 * (1 - done) * val[1:] - val[:-1]
    assert rel_err(adv.cpu().numpy(), td) < 1e-6


# ---------------------------------------------------------------- Adam
def test_adam_parity(P):
    say("adam")
    g = np.random.default_rng(0)
    n = 100_003
    th = (0.05 * g.standard_normal(n)).astype(np.float32)   # weight-sized values
    master = torch.tensor(th, device=DEV)
    lp = torch.empty(n, dtype=torch.bfloat16, device=DEV)
    opt = P.Adam(n, DEV, lr=2.5e-4)
    tho, m, v = th.astype(np.float64), np.zeros(n), np.zeros(n)
    for k in range(1, 4):
        gr = g.standard_normal(n).astype(np.float32) * (10.0 ** g.uniform(-3, 1, n)).astype(np.float32)
        before = master.cpu().numpy().astype(np.float64)
        opt.step(master, torch.tensor(gr, device=DEV), lp)
        tho, m, v = ppo.adam(before, gr.astype(np.float64), m, v, k, 2.5e-4)
        got = master.cpu().numpy().astype(np.float64)
        # float32 storage of theta bounds the agreement of the update
        assert rel_err(got - before, tho - before) < 1e-4
    st = opt.state()
    assert st["step"] == 3 and st["skipped"] == 0
    assert torch.equal(lp, master.to(torch.bfloat16))


def test_adam_skips_non_finite_and_halves_scale(P):
    n = 4099
    master = torch.randn(n, device=DEV)
    opt = P.Adam(n, DEV, lr=1e-3, loss_scale=1024.0, growth_interval=2)
    g = torch.randn(n, device=DEV) * 1024
    opt.step(master, g)
    m0, v0, th0 = opt.m.clone(), opt.v.clone(), master.clone()
    g[17] = float("inf")
    opt.step(master, g)
    st = opt.state()
    assert torch.equal(master, th0) and torch.equal(opt.m, m0) and torch.equal(opt.v, v0)
    assert st["scale"] == 512.0 and st["step"] == 1 and st["skipped"] == 1 and st["found_inf"] == 1
    g[17] = 0.0
    opt.step(master, g)
    opt.step(master, g)
    assert opt.state()["scale"] == 1024.0 and opt.state()["step"] == 3


# ---------------------------------------------------------------- act
def _act_case(P, net, dtype, B, seed, state_rows=0):
    flat = R.init_params(net, seed, random_affine=True)
    g = np.random.default_rng(seed + 100)
    obs = g.random((B, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32)
    if dtype == "bf16":
        obs = R.round_bf16(obs)
    goal = g.standard_normal((B, 2)).astype(np.float32)
    prev = g.integers(0, net.num_actions, B).astype(np.int32)
    mask = (g.random(B) > 0.3).astype(np.float32)
    SR = state_rows or B
    h = (0.5 * g.standard_normal((net.lstm_layers, SR, net.hidden))).astype(np.float32)
    c = (0.5 * g.standard_normal((net.lstm_layers, SR, net.hidden))).astype(np.float32)
    u = g.random(B).astype(np.float32)
    n = P.Net(net, dtype)
    params = torch.tensor(flat, device=DEV)
    lp = P.cast_bf16(params) if dtype == "bf16" else None
    td = lambda a: torch.tensor(a, device=DEV)
    h_in, c_in = td(h), td(c)
    out = n.act(td(obs).to(torch.bfloat16) if dtype == "bf16" else td(obs), td(goal), td(prev), td(mask),
                h_in, c_in, td(u), params, lp, want_logits=True, state_rows=SR)
    torch.cuda.synchronize()
    ref = policy.act(OP.unpack(net, flat), net, obs, goal, prev, mask, h[:, :B], c[:, :B], u)
    ref["u"] = u
    return out, ref


@pytest.mark.parametrize("name,net,dtype,B", [("tiny", TINY_NET, "f32", 2), ("tiny", TINY_NET, "f32", 5),
                                              ("tiny+", TINY_PLUS, "f32", 3),
                                              ("mini_resnet", MINI_RESNET, "f32", 4),
                                              ("resnet_smallcore", RESNET_SMALLCORE, "f32", 2),
                                              ("tiny_bigcore", TINY_BIGCORE, "f32", 4),
                                              ("tiny_core1024", TINY_CORE1024, "f32", 3),
                                              ("tiny_core1024", TINY_CORE1024, "bf16", 3),
                                              ("resnet64", RESNET_64, "f32", 2),
                                              ("tiny+", TINY_PLUS, "bf16", 3),
                                              ("mini_resnet", MINI_RESNET, "bf16", 4)])
def test_act_parity_small(P, name, net, dtype, B):
    say(f"act {name} {dtype} B={B}")
    out, ref = _act_case(P, net, dtype, B, seed=B)
    tol = TOL[dtype]
    assert rel_err(out["logits"].cpu().numpy(), ref["logits"]) < tol
    assert rel_err(out["value"].cpu().numpy(), ref["value"]) < tol
    assert rel_err(out["h"].cpu().numpy(), ref["h"]) < tol
    assert rel_err(out["c"].cpu().numpy(), ref["c"]) < tol
    if dtype == "f32":
        np.testing.assert_array_equal(out["action"].cpu().numpy(), ref["action"])
        assert rel_err(out["logp"].cpu().numpy(), ref["logp"]) < tol


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_act_parity_resnet_paper_shape(P, dtype):
    """The paper's encoder at 256x256 frames, batch 4 (one act step of a worker)."""
    say(f"act resnet {dtype}")
    out, ref = _act_case(P, C1.net, dtype, 4, seed=11, state_rows=6)
    tol = TOL[dtype]
    assert rel_err(out["logits"].cpu().numpy(), ref["logits"]) < tol
    assert rel_err(out["value"].cpu().numpy(), ref["value"]) < tol
    assert rel_err(out["h"].cpu().numpy()[:, :4], ref["h"]) < tol
    assert_actions_agree(out["action"].cpu().numpy(), ref, tol)


def assert_actions_agree(a, ref, tol):
    """Identical actions, or a flip explained by the logit error: u lies
    within tol of the cumulative probability at the boundary between them."""
    ar = ref["action"]
    p = np.exp(ref["logits"] - ref["logits"].max(1, keepdims=True))
    p /= p.sum(1, keepdims=True)
    cdf = np.cumsum(p, 1)
    for i in np.nonzero(a != ar)[0]:
        k = min(a[i], ar[i])
        assert abs(ref["u"][i] - cdf[i, k]) < tol, (i, a[i], ar[i], ref["u"][i], cdf[i])


# ---------------------------------------------------------- loss backward
def gpu_decisions(n, net, F, nb, mb):
    """The ReLU patterns and max-pool winners the GPU used in its last
    ppo_loss_backward, in the oracle's layout (frames time-major)."""
    from paper_1911_00357_amd._lib import PPO_OP_LEARN
    ws = n.last_workspace(PPO_OP_LEARN)
    dec = {}
    nunits = n.probe(PPO_OP_LEARN, F, nb, 3)[3][0]
    for i in range(nunits):
        name, relu, off, (ho, wo, C, chw) = n.probe(PPO_OP_LEARN, F, nb, 0, i)
        if not relu:
            continue
        a = ws[off:off + F * ho * wo * C * 4].view(torch.float32).cpu().numpy()
        a = a.reshape(F, C, ho, wo) if chw else a.reshape(F, ho, wo, C).transpose(0, 3, 1, 2)
        key = name[len("enc."):]
        if key.endswith(".c3"):
            key = key[:-2] + "out"
        dec[key] = a > 0
    if net.trunk == "resnet":
        _, _, off, (h, w, C, _) = n.probe(PPO_OP_LEARN, F, nb, 1)
        dec["maxpool"] = ws[off:off + F * h * w * C].cpu().numpy().reshape(F, h, w, C).transpose(0, 3, 1, 2)
    _, _, off, (d0, vis, _, _) = n.probe(PPO_OP_LEARN, F, nb, 2)
    z = ws[off:off + F * d0 * 4].view(torch.float32).cpu().numpy().reshape(F, d0)
    TB, B = mb["action"].shape
    valid = np.arange(TB)[:, None] < mb["lens"][None, :]
    tt, jj = np.nonzero(valid)
    vm = np.zeros((TB, B, vis), bool)
    vm[tt, jj] = z[:, :vis] > 0
    dec["vis"] = vm
    return dec


def _loss_case(P, net, dtype, T, N, envs, lengths, seed, norm_adv=False, same_decisions=False):
    flat = R.init_params(net, seed, random_affine=True)
    rec = random_record(net, T, N, seed + 1, lengths=lengths, bf16=dtype == "bf16")
    if lengths is not None:   # longest first (the library's packing order)
        envs = sorted(envs, key=lambda e: -lengths[e])
    n = P.Net(net, dtype)
    params = torch.tensor(flat, device=DEV)
    lp = P.cast_bf16(params) if dtype == "bf16" else None
    ro = to_device(rec, bf16=dtype == "bf16")
    adv_stats = None
    mu_var = None
    if norm_adv:
        mu_var = ppo.adv_stats(rec["adv"].astype(np.float64), rec["lengths"])
        adv_stats = torch.tensor(np.array(mu_var), dtype=torch.float64, device=DEV)
    cfg = P.LossCfg(norm_adv=norm_adv)
    grad, stats = n.loss_backward(ro, envs, rec["lengths"] if lengths is not None else None, params, lp, cfg,
                                  loss_scale=torch.tensor([1.0], device=DEV), adv_stats=adv_stats)
    torch.cuda.synchronize()
    mb = oracle_minibatch(rec, envs)
    dec = None
    if same_decisions:
        F = int(mb["lens"].sum())
        dec = gpu_decisions(n, net, F, len(envs), mb)
    s_ref, g_ref = ppo.loss_grad(flat.astype(np.float64), net, PPOCfg(), mb, adv_norm=mu_var, decide=dec)
    floor = None
    if dtype == "bf16" and same_decisions:
        # the exact gradient at the bfloat16-rounded weights, same decisions: how far
        # rounding the working copy alone moves each tensor's gradient
        _, g_w = ppo.loss_grad(R.round_bf16(flat).astype(np.float64), net, PPOCfg(), mb, adv_norm=mu_var,
                               decide=dec)
        floor = per_tensor_errors(net, g_w, g_ref)
    return grad.cpu().numpy(), stats.cpu().numpy(), g_ref, s_ref, floor


def check_loss(net, dtype, g, s, g_ref, s_ref, tag, floor=None):
    """Loss terms and the whole gradient within the tolerance; each parameter
    tensor's gradient within the tolerance, or (bfloat16) within 4x the change
    that rounding the weights to bfloat16 alone causes in the exact gradient
    (cancellation-heavy tensors such as deep GroupNorm scales).  The kernels
    round both operands of every product (weights and activations) and the
    floor measures the weight rounding only: about twice the floor is the
    expected error, and the bound leaves a factor 2 over that."""
    tol = TOL[dtype]
    errs = per_tensor_errors(net, g, g_ref)
    order = sorted(errs, key=errs.get, reverse=True)
    say(f"  {tag}: global grad err {rel_err(g, g_ref):.2e}; worst tensors: " +
        ", ".join(f"{k}={errs[k]:.1e}" + (f"(floor {floor[k]:.1e})" if floor else "") for k in order[:5]) +
        f"; loss {s[0]:.6f} vs {s_ref[0]:.6f}")
    denom = abs(s_ref[1]) + 0.5 * abs(s_ref[2]) + 0.01 * abs(s_ref[3])
    assert abs(s[0] - s_ref[0]) / denom < tol
    for k in (1, 2, 3):
        assert abs(s[k] - s_ref[k]) <= tol * max(abs(s_ref[k]), 1e-6)
    assert rel_err(g, g_ref) < tol
    bad = {k: v for k, v in errs.items() if v >= tol and (floor is None or v >= 4 * floor[k])}
    assert not bad, bad


@pytest.mark.parametrize("name,net,T,N,envs,lengths", [
    ("tiny", TINY_NET, 16, 2, [0, 1], None),
    ("tiny_ragged", TINY_NET, 9, 4, [3, 0, 2], [9, 4, 7, 2]),
    ("tiny+", TINY_PLUS, 6, 3, [0, 2], [6, 5, 3]),
    ("mini_resnet", MINI_RESNET, 5, 3, [2, 1, 0], [5, 3, 4]),
])
def test_loss_backward_parity_f32(P, name, net, T, N, envs, lengths):
    say(f"loss f32 {name}")
    g, s, g_ref, s_ref, _ = _loss_case(P, net, "f32", T, N, envs, lengths, seed=T * 7 + N)
    check_loss(net, "f32", g, s, g_ref, s_ref, name)


def test_loss_backward_norm_adv(P):
    g, s, g_ref, s_ref, _ = _loss_case(P, TINY_PLUS, "f32", 5, 3, [0, 1, 2], None, seed=3, norm_adv=True)
    assert rel_err(g, g_ref) < 1e-4 and abs(s[1] - s_ref[1]) < 1e-4 * abs(s_ref[1])


@pytest.mark.parametrize("name,net,T,N,envs,lengths", [
    ("tiny+", TINY_PLUS, 6, 3, [0, 2], [6, 5, 3]),
    ("mini_resnet", MINI_RESNET, 5, 3, [2, 1, 0], [5, 3, 4]),
])
def test_loss_backward_parity_bf16(P, name, net, T, N, envs, lengths):
    """bfloat16 operands move activations across ReLU kinks; the oracle takes
    the GPU's ReLU / max-pool decisions."""
    say(f"loss bf16 {name}")
    g, s, g_ref, s_ref, floor = _loss_case(P, net, "bf16", T, N, envs, lengths, seed=T * 3 + N,
                                           same_decisions=True)
    check_loss(net, "bf16", g, s, g_ref, s_ref, name, floor)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_loss_backward_resnet_paper_shape(P, dtype):
    """The paper's network at 256x256 frames: 2 envs x (4, 3) steps.  The
    oracle takes the GPU's ReLU / max-pool decisions (a decision made by
    floating point is taken in the kernel's precision on both sides)."""
    say(f"loss resnet paper shape {dtype}")
    g, s, g_ref, s_ref, floor = _loss_case(P, C1.net, dtype, 4, 3, [2, 0], [4, 2, 3], seed=21,
                                           same_decisions=True)
    check_loss(C1.net, dtype, g, s, g_ref, s_ref, "resnet", floor)


@pytest.mark.parametrize("limit", ["0", "1000000000"], ids=["partial_finalize_apply", "one_launch"])
def test_loss_backward_both_groupnorm_forms(P, limit, monkeypatch):
    """Both GroupNorm forms (per image-and-group launch; coalesced partial /
    finalize / apply) against the oracle on the same case."""
    monkeypatch.setenv("DDPPO_GN_FUSED_MAX", limit)
    say(f"loss f32 mini_resnet, GroupNorm form limit {limit}")
    g, s, g_ref, s_ref, _ = _loss_case(P, MINI_RESNET, "f32", 5, 3, [2, 1, 0], [5, 3, 4], seed=38)
    check_loss(MINI_RESNET, "f32", g, s, g_ref, s_ref, f"mini_resnet gn limit {limit}")


def test_autotuned_loss_backward(P):
    """The tile autotuner: the tuning call and a later call from the table give
    the same bits, both within the tolerance of the oracle."""
    say("autotuned loss backward")
    net, T, N, envs, lengths = MINI_RESNET, 5, 3, [2, 1, 0], [5, 3, 4]
    flat = R.init_params(net, 41, random_affine=True)
    rec = random_record(net, T, N, 42, lengths=lengths)
    envs = sorted(envs, key=lambda e: -lengths[e])
    n = P.Net(net, "f32")
    params = torch.tensor(flat, device=DEV)
    ro = to_device(rec)
    n.autotune(1)
    g1, s1 = n.loss_backward(ro, envs, rec["lengths"], params, None, P.LossCfg(),
                             loss_scale=torch.tensor([1.0], device=DEV))
    entries = n.autotune(0)
    g2, s2 = n.loss_backward(ro, envs, rec["lengths"], params, None, P.LossCfg(),
                             loss_scale=torch.tensor([1.0], device=DEV))
    torch.cuda.synchronize()
    assert entries > 0
    assert torch.equal(g1, g2) and torch.equal(s1, s2)
    mb = oracle_minibatch(rec, envs)
    s_ref, g_ref = ppo.loss_grad(flat.astype(np.float64), net, PPOCfg(), mb)
    assert rel_err(g2.cpu().numpy(), g_ref) < 1e-4
    assert n.autotune(-1) == 0


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_autotuned_act(P, dtype):
    """Act calls whose convolutions leave split-K partials for the GroupNorm
    take tuned tiles too: the tuning call and a later call from the table give
    the same bits, within the tolerance of the oracle."""
    say(f"autotuned act {dtype}")
    net, B = C1.net, 4
    flat = R.init_params(net, 23, random_affine=True)
    g = np.random.default_rng(24)
    obs = g.random((B, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32)
    if dtype == "bf16":
        obs = R.round_bf16(obs)
    goal = g.standard_normal((B, 2)).astype(np.float32)
    prev = g.integers(0, net.num_actions, B).astype(np.int32)
    mask = np.ones(B, np.float32)
    h = (0.5 * g.standard_normal((net.lstm_layers, B, net.hidden))).astype(np.float32)
    c = (0.5 * g.standard_normal((net.lstm_layers, B, net.hidden))).astype(np.float32)
    u = g.random(B).astype(np.float32)
    n = P.Net(net, dtype)
    params = torch.tensor(flat, device=DEV)
    lp = P.cast_bf16(params) if dtype == "bf16" else None
    td = lambda a: torch.tensor(a, device=DEV)
    o = td(obs).to(torch.bfloat16) if dtype == "bf16" else td(obs)
    n.autotune(1)
    out1 = n.act(o, td(goal), td(prev), td(mask), td(h), td(c), td(u), params, lp, want_logits=True)
    entries = n.autotune(0)
    out2 = n.act(o, td(goal), td(prev), td(mask), td(h), td(c), td(u), params, lp, want_logits=True)
    torch.cuda.synchronize()
    assert entries > 0
    for k in ("logits", "value", "h", "c", "action"):
        assert torch.equal(out1[k], out2[k]), k
    ref = policy.act(OP.unpack(net, flat), net, obs, goal, prev, mask, h, c, u)
    ref["u"] = u
    tol = TOL[dtype]
    assert rel_err(out2["logits"].cpu().numpy(), ref["logits"]) < tol
    assert rel_err(out2["h"].cpu().numpy(), ref["h"]) < tol
    assert_actions_agree(out2["action"].cpu().numpy(), ref, tol)
