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
from synth.configs import C0, C1, SERESNEXT_NET, PPOCfg
from tests.gpu_util import (DEV, assert_close, errs, flip_summary, oracle_minibatch, random_record, rel_err,
                            tensor_errors, to_device, validate_decisions)
from tests.nets import (MINI_RESNET, MINI_SERESNEXT, RESNET_64, RESNET_SMALLCORE, TINY_BIGCORE, TINY_CORE1024,
                        TINY_NET, TINY_PLUS)

pytestmark = pytest.mark.gpu
TOL = {"f32": 1e-4, "bf16": 2e-2}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ---------------------------------------------------------------- GAE
@pytest.mark.parametrize("T,N,ragged,seed", [(16, 2, False, 0), (128, 4, False, 1), (128, 64, True, 2),
                                             (1, 3, False, 3), (200, 5, True, 4), (64, 1, False, 5),
                                             (70, 130, True, 6), (65, 64, False, 7)])
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
    assert_close("advantages", adv.cpu().numpy(), A, 1e-5)
    assert_close("returns", ret.cpu().numpy(), Rt, 1e-5)
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
    assert_close("advantages", adv.cpu().numpy(), td, 1e-6)


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
        assert_close("update", got - before, tho - before, 1e-4)
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


def test_adam_static_scale_kept_on_skip(P):
    """A float32 net's scale (1, no growth) stays 1 when a non-finite gradient
    skips a step, so later gradients are not rescaled."""
    n = 1000
    master = torch.randn(n, device=DEV)
    opt = P.Adam(n, DEV, lr=1e-3, loss_scale=1.0, growth_interval=0)
    g = torch.randn(n, device=DEV)
    g[3] = float("nan")
    th0 = master.clone()
    opt.step(master, g)
    st = opt.state()
    assert torch.equal(master, th0) and st["skipped"] == 1 and st["scale"] == 1.0 and st["step"] == 0
    g[3] = 0.0
    opt.step(master, g)
    tho, _, _ = ppo.adam(th0.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64),
                         np.zeros(n), np.zeros(n), 1, 1e-3)
    assert opt.state()["scale"] == 1.0 and opt.state()["step"] == 1
    assert_close("update", master.cpu().numpy() - th0.cpu().numpy(), tho - th0.cpu().numpy(), 1e-4)


# ---------------------------------------------------------------- act
def _act_case(P, net, dtype, B, seed, state_rows=0, mask=None, u=None):
    flat = R.init_params(net, seed, random_affine=True)
    g = np.random.default_rng(seed + 100)
    obs = g.random((B, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32)
    if dtype == "bf16":
        obs = R.round_bf16(obs)
    goal = g.standard_normal((B, 2)).astype(np.float32)
    prev = g.integers(0, net.num_actions, B).astype(np.int32)
    rmask = (g.random(B) > 0.3).astype(np.float32)
    mask = rmask if mask is None else np.full(B, mask, np.float32)
    SR = state_rows or B
    h = (0.5 * g.standard_normal((net.lstm_layers, SR, net.hidden))).astype(np.float32)
    c = (0.5 * g.standard_normal((net.lstm_layers, SR, net.hidden))).astype(np.float32)
    ru = g.random(B).astype(np.float32)
    u = ru if u is None else np.full(B, u, np.float32)
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
    if dtype == "bf16":
        ref["form"] = policy.act(OP.unpack(net, flat), net, obs, goal, prev, mask, h[:, :B], c[:, :B], u,
                                 quant="bf16")
        ref["form"]["u"] = u
    return out, ref


def check_act(out, ref, dtype, B, tag):
    """Logits, value, h, c (and float32 log-probs) within the tolerance of the
    float64 oracle (relative L2 and element-wise); float32 actions identical,
    bfloat16 actions identical or flipped only where u lies within the
    tolerance of a CDF step.  For bfloat16 the error of the oracle's own
    bfloat16 precision form is printed beside the GPU's (a forward pass is
    continuous: no decision is imposed)."""
    tol = TOL[dtype]
    g = lambda k: out[k].cpu().numpy()[:, :B] if k in ("h", "c") else out[k].cpu().numpy()
    line = []
    for k in ("logits", "value", "h", "c"):
        l2, mx = assert_close(k, g(k), ref[k], tol)
        line.append(f"{k} {l2:.1e}/{mx:.1e}")
        if dtype == "bf16":
            line[-1] += " (form %.1e/%.1e)" % errs(ref["form"][k], ref[k])
    say(f"  {tag}: " + "; ".join(line))
    if dtype == "f32":
        np.testing.assert_array_equal(g("action"), ref["action"])
        assert_close("logp", g("logp"), ref["logp"], tol)
    else:
        assert_actions_agree(g("action"), ref, tol)


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
    check_act(out, ref, dtype, B, name)


@pytest.mark.parametrize("name,net,dtype,B,mask,u", [
    ("tiny", TINY_NET, "f32", 1, 0.0, None),                     # one env, an episode start
    ("mini_resnet", MINI_RESNET, "f32", 1, 1.0, 0.0),            # u = 0: the first action
    ("mini_resnet", MINI_RESNET, "f32", 3, 0.0, 0.99999994),     # u just below 1: the last CDF step
    ("tiny+", TINY_PLUS, "bf16", 2, 0.0, 0.0),
])
def test_act_parity_degenerate(P, name, net, dtype, B, mask, u):
    """A single env, every row an episode start (the state zeroed, the
    start-token embedding), and the sample's extreme uniforms."""
    say(f"act degenerate {name} {dtype} B={B} mask={mask} u={u}")
    out, ref = _act_case(P, net, dtype, B, seed=40 + B, mask=mask, u=u)
    check_act(out, ref, dtype, B, name)
    if u == 0.0:
        assert (out["action"].cpu().numpy() == ref["action"]).all()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_act_parity_resnet_paper_shape(P, dtype):
    """The paper's encoder at 256x256 frames, batch 4 (one act step of a worker)."""
    say(f"act resnet {dtype}")
    out, ref = _act_case(P, C1.net, dtype, 4, seed=11, state_rows=6)
    check_act(out, ref, dtype, 4, "resnet")


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
def _ws_f32(ws, off, n):
    return ws[off:off + n * 4].view(torch.float32).cpu().numpy()


def gpu_decisions(n, net, F, nb, mb, codes=False):
    """The ReLU patterns and max-pool winners the GPU used in its last
    learner call, in the oracle's layout (frames time-major); with codes,
    also the bfloat16 codes of every activation operand it rounded (each
    convolution's input by the convolution's name, the visual FC's input, each
    LSTM layer's input and masked previous state), as decide's 'q:' keys."""
    from oracle.nn import round_bf16
    from paper_1911_00357_amd._lib import PPO_OP_LEARN
    ws = n.last_workspace(PPO_OP_LEARN)
    dec = {}
    nunits = n.probe(PPO_OP_LEARN, F, nb, 3)[3][0]
    outs = {}
    for i in range(nunits):
        name, relu, off, (ho, wo, C, chw) = n.probe(PPO_OP_LEARN, F, nb, 0, i)
        if not relu and not codes:
            continue
        a = _ws_f32(ws, off, F * ho * wo * C)
        a = a.reshape(F, C, ho, wo) if chw else a.reshape(F, ho, wo, C).transpose(0, 3, 1, 2)
        key = name[len("enc."):]
        if relu:
            dec[key[:-2] + "out" if key.endswith(".c3") else key] = a > 0
        if codes:
            outs[key] = round_bf16(a)
    if net.trunk != "tiny":
        _, _, off, (h, w, C, _) = n.probe(PPO_OP_LEARN, F, nb, 1)
        dec["maxpool"] = ws[off:off + F * h * w * C].cpu().numpy().reshape(F, h, w, C).transpose(0, 3, 1, 2)
    if net.trunk == "seresnext":          # each block's squeeze-excite hidden ReLU
        bi = 0
        for s_ in range(4):
            for j in range(net.blocks[s_]):
                _, _, off, (R, _, _, _) = n.probe(PPO_OP_LEARN, F, nb, 8, bi)
                dec["s%d.b%d.se" % (s_, j)] = _ws_f32(ws, off, F * R).reshape(F, R) > 0
                bi += 1
    TB, B = mb["action"].shape
    valid = np.arange(TB)[:, None] < mb["lens"][None, :]
    tt, jj = np.nonzero(valid)

    def tm(rows):                       # packed frame rows -> [T_B, B, .] (invalid frames 0)
        o = np.zeros((TB, B) + rows.shape[1:], rows.dtype)
        o[tt, jj] = rows
        return o

    _, _, off, (d0, vis, _, _) = n.probe(PPO_OP_LEARN, F, nb, 2)
    z = _ws_f32(ws, off, F * d0).reshape(F, d0)
    dec["vis"] = tm(z[:, :vis] > 0)
    if codes:
        if net.trunk != "tiny":
            _, _, off, (h, w, C, _) = n.probe(PPO_OP_LEARN, F, nb, 5)
            prev = round_bf16(_ws_f32(ws, off, F * h * w * C).reshape(F, h, w, C).transpose(0, 3, 1, 2))
            for s_ in range(4):
                for j in range(net.blocks[s_]):
                    pre = "s%d.b%d." % (s_, j)
                    dec["q:" + pre + "c1"] = prev
                    if j == 0:
                        dec["q:" + pre + "ds"] = prev
                    dec["q:" + pre + "c2"] = outs[pre + "c1"]
                    dec["q:" + pre + "c3"] = outs[pre + "c2"]
                    prev = outs[pre + "c3"]
            dec["q:compress"] = prev
            last = outs["compress"]
        else:
            dec["q:conv2"] = outs["conv1"]
            last = outs["conv2"]
        dec["q:fc"] = tm(last.reshape(F, -1))
        dec["q:lstm0.x"] = tm(round_bf16(z))
        H = net.hidden
        for l in range(net.lstm_layers):
            off = n.probe(PPO_OP_LEARN, F, nb, 6, l)[2]
            dec["q:lstm%d.h" % l] = tm(round_bf16(_ws_f32(ws, off, F * H).reshape(F, H)))
            if l + 1 < net.lstm_layers:
                off = n.probe(PPO_OP_LEARN, F, nb, 7, l)[2]
                dec["q:lstm%d.x" % (l + 1)] = tm(round_bf16(_ws_f32(ws, off, F * H).reshape(F, H)))
    return dec


FLIP_TOL = {"f32": 1e-3, "bf16": 1e-3}     # near-kink margin of a flipped decision (x rms)
QTOL = 1e-4      # an imposed bfloat16 code: the rounding of a value within QTOL x rms of the oracle's
AT_RISK = 1e-2   # bfloat16 tensors whose precision-form error (own rounding) reaches this are reported


class LossCase:
    """GPU loss/gradient of one minibatch (g, s) and its oracle references,
    with the GPU's ReLU / max-pool decisions imposed when `flips` is set:
    `exact` (float64); for bfloat16 also `own` (the precision form with its
    own roundings: the form's cost) and `form` (the precision form with the
    GPU's bfloat16 operand codes imposed too: what the kernels must match)."""


def oracle_refs(c, net, dtype, flat, mb, dec, mu_var=None, coded=None):
    """Fill c's oracle references (see LossCase); dec: the GPU's decisions,
    coded: the same plus operand codes (bfloat16)."""
    flat64 = flat.astype(np.float64)
    cfg = PPOCfg()
    r = {} if dec is not None else None
    if dtype == "f32":
        c.s_exact, c.g_exact = ppo.loss_grad(flat64, net, cfg, mb, adv_norm=mu_var, decide=dec, record=r,
                                             record_outputs=False)
        if dec is not None:
            c.flips = validate_decisions(dec, r, mb["lens"], FLIP_TOL[dtype])
        return c
    c.s_form, c.g_form = ppo.loss_grad(flat64, net, cfg, mb, adv_norm=mu_var, decide=coded, quant="bf16",
                                       record=r, record_outputs=False)
    if coded is not None:
        c.flips = validate_decisions(coded, r, mb["lens"], FLIP_TOL[dtype], QTOL)
    del r
    c.s_own, c.g_own = ppo.loss_grad(flat64, net, cfg, mb, adv_norm=mu_var, decide=dec, quant="bf16")
    c.s_exact, c.g_exact = ppo.loss_grad(flat64, net, cfg, mb, adv_norm=mu_var, decide=dec)
    return c


def _loss_case(P, net, dtype, T, N, envs, lengths, seed, norm_adv=False, same_decisions=False, rec=None):
    flat = R.init_params(net, seed, random_affine=True)
    rec = rec or random_record(net, T, N, seed + 1, lengths=lengths, bf16=dtype == "bf16")
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
    c = LossCase()
    c.g, c.s = grad.cpu().numpy(), stats.cpu().numpy()
    c.flips = None
    dec = coded = None
    if same_decisions:
        F = int(mb["lens"].sum())
        if dtype == "bf16":
            coded = gpu_decisions(n, net, F, len(envs), mb, codes=True)
            dec = {k: v for k, v in coded.items() if not k.startswith("q:")}
        else:
            dec = gpu_decisions(n, net, F, len(envs), mb)
    del n, ro
    torch.cuda.empty_cache()
    return oracle_refs(c, net, dtype, flat, mb, dec, mu_var, coded)


def _loss_rel(s, s_ref):
    """Loss terms' errors: total relative to |L_pg| + c_v |L_v| + c_e |L_H|,
    each term relative to itself."""
    denom = abs(s_ref[1]) + 0.5 * abs(s_ref[2]) + 0.01 * abs(s_ref[3])
    return [abs(s[0] - s_ref[0]) / denom] + [abs(s[k] - s_ref[k]) / max(abs(s_ref[k]), 1e-6) for k in (1, 2, 3)]


def check_loss(net, dtype, c, tag):
    """float32: every loss term, the whole gradient and each parameter
    tensor's gradient (relative L2 and element-wise) within 1e-4 of the
    float64 oracle.

    bfloat16: (i) against the bfloat16 precision form with the GPU's
    decisions and operand codes imposed (so both sides multiply the same
    operands): loss terms within 1e-4, the whole gradient within 1e-3 and each
    tensor within 5e-3 (relative L2 and element-wise) -- the kernels' gradient
    operands carry 16 significant bits (hi + lo), 2^7 times float32's
    rounding, and the float32 path's worst tensors sit near 3e-5;
    (ii) against the float64 oracle (the GPU's decisions imposed): loss terms
    and the whole gradient within 2e-2, and each tensor within 2e-2 except
    tensors on which the form with its own roundings already reaches 1e-2
    (its error there is one draw of the rounding noise, the GPU's another);
    those are listed with both errors."""
    tol = TOL[dtype]
    er = tensor_errors(net, c.g, c.g_exact)
    order = sorted(er, key=lambda k: -er[k][0])
    say(f"  {tag}: grad err {rel_err(c.g, c.g_exact):.2e}; worst tensors (L2, elem): " +
        ", ".join(f"{k}=({er[k][0]:.1e},{er[k][1]:.1e})" for k in order[:4]) +
        f"; loss {c.s[0]:.6f} vs {c.s_exact[0]:.6f}" +
        (f"; {flip_summary(c.flips)}" if c.flips is not None else ""))
    at_risk = {}
    if dtype == "bf16":
        eq = tensor_errors(net, c.g, c.g_form)
        worst = sorted(eq, key=lambda k: -max(eq[k]))[:4]
        say(f"  {tag}: vs bf16 form with the GPU's codes: grad {rel_err(c.g, c.g_form):.2e}, loss "
            f"{max(_loss_rel(c.s, c.s_form)):.1e}; worst tensors " +
            ", ".join(f"{k}=({eq[k][0]:.1e},{eq[k][1]:.1e})" for k in worst))
        assert max(_loss_rel(c.s, c.s_form)) < 1e-4
        assert rel_err(c.g, c.g_form) < 1e-3
        bad = {k: eq[k] for k in eq if max(eq[k]) >= 5e-3}
        assert not bad, f"GPU vs bf16 form (L2, elem): {bad}"
        eo = tensor_errors(net, c.g_own, c.g_exact)
        at_risk = {k: eo[k] for k in eo if max(eo[k]) >= AT_RISK}
        over = {k: er[k] for k in at_risk if max(er[k]) >= tol}
        say(f"  {tag}: bf16 form (own roundings) vs exact: grad {rel_err(c.g_own, c.g_exact):.2e}; "
            f"{len(at_risk)} tensors at risk (form error >= {AT_RISK:.0e}), {len(over)} of them over {tol:.0e} on "
            f"the GPU" + ("".join(f"; {k}: form ({eo[k][0]:.1e},{eo[k][1]:.1e}), GPU ({er[k][0]:.1e},"
                                  f"{er[k][1]:.1e})" for k in over)))
    assert max(_loss_rel(c.s, c.s_exact)) < tol
    assert_close("gradient", c.g, c.g_exact, tol)
    bad = {k: er[k] for k in er if max(er[k]) >= tol and k not in at_risk}
    assert not bad, bad


@pytest.mark.parametrize("name,net,T,N,envs,lengths", [
    ("tiny", TINY_NET, 16, 2, [0, 1], None),
    ("tiny_ragged", TINY_NET, 9, 4, [3, 0, 2], [9, 4, 7, 2]),
    ("tiny+", TINY_PLUS, 6, 3, [0, 2], [6, 5, 3]),
    ("mini_resnet", MINI_RESNET, 5, 3, [2, 1, 0], [5, 3, 4]),
    ("tiny_one_frame", TINY_NET, 5, 3, [1], [5, 1, 3]),          # one env of length 1: a single frame
    ("tiny_one_env", TINY_NET, 4, 1, [0], None),
])
def test_loss_backward_parity_f32(P, name, net, T, N, envs, lengths):
    say(f"loss f32 {name}")
    c = _loss_case(P, net, "f32", T, N, envs, lengths, seed=T * 7 + N, same_decisions=True)
    check_loss(net, "f32", c, name)


def test_loss_backward_norm_adv(P):
    say("loss f32 tiny+ norm_adv")
    c = _loss_case(P, TINY_PLUS, "f32", 5, 3, [0, 1, 2], None, seed=3, norm_adv=True, same_decisions=True)
    check_loss(TINY_PLUS, "f32", c, "tiny+ norm_adv")


@pytest.mark.parametrize("name,net,T,N,envs,lengths", [
    ("tiny+", TINY_PLUS, 6, 3, [0, 2], [6, 5, 3]),
    ("mini_resnet", MINI_RESNET, 5, 3, [2, 1, 0], [5, 3, 4]),
])
def test_loss_backward_parity_bf16(P, name, net, T, N, envs, lengths):
    """bfloat16 operands move activations across ReLU kinks; the oracle takes
    the GPU's ReLU / max-pool decisions, each checked to sit at a near-kink."""
    say(f"loss bf16 {name}")
    c = _loss_case(P, net, "bf16", T, N, envs, lengths, seed=T * 3 + N, same_decisions=True)
    check_loss(net, "bf16", c, name)


# GroupNorm form limits (elements per tensor below which one launch per
# (image, group) is used): "0" forces the coalesced partial / finalize /
# apply kernels of learner-size tensors, a large value the one-launch form
GN_FORMS = {"partial": {"DDPPO_GN_FUSED_MAX": "0", "DDPPO_GNB_FUSED_MAX": "0"},
            "one_launch": {"DDPPO_GN_FUSED_MAX": "1000000000", "DDPPO_GNB_FUSED_MAX": "1000000000"},
            "default": {}}


@pytest.mark.parametrize("form", ["default", "partial"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_loss_backward_resnet_paper_shape(P, dtype, form, monkeypatch):
    """The paper's network at 256x256 frames: 2 envs x (4, 3) steps, in the
    default GroupNorm choice and with the learner-size GroupNorm kernels
    (forward and backward partial forms at full width) forced.  The oracle
    takes the GPU's ReLU / max-pool decisions (a decision made by floating
    point is taken in the kernel's precision on both sides)."""
    for k, v in GN_FORMS[form].items():
        monkeypatch.setenv(k, v)
    say(f"loss resnet paper shape {dtype}, GroupNorm {form}")
    c = _loss_case(P, C1.net, dtype, 4, 3, [2, 0], [4, 2, 3], seed=21, same_decisions=True)
    check_loss(C1.net, dtype, c, f"resnet {form}")


@pytest.mark.parametrize("form", ["partial", "one_launch"])
def test_loss_backward_both_groupnorm_forms(P, form, monkeypatch):
    """Both GroupNorm forms (per image-and-group launch; coalesced partial /
    finalize / apply, forward and backward) against the oracle on the same case."""
    for k, v in GN_FORMS[form].items():
        monkeypatch.setenv(k, v)
    say(f"loss f32 mini_resnet, GroupNorm {form}")
    c = _loss_case(P, MINI_RESNET, "f32", 5, 3, [2, 1, 0], [5, 3, 4], seed=38, same_decisions=True)
    check_loss(MINI_RESNET, "f32", c, f"mini_resnet gn {form}")


def test_loss_backward_worker_minibatch_f32(P):
    """One minibatch at the paper worker's learner size: 2 envs x T=128 at
    256x256 (256 frames), the tile / split choices and the 128-step
    recurrence the benchmark runs; every frame checked through the oracle."""
    say("loss f32 resnet, 2 envs x T=128 (256 frames)")
    c = _loss_case(P, C1.net, "f32", 128, 2, [1, 0], None, seed=51, same_decisions=True)
    check_loss(C1.net, "f32", c, "resnet 256 frames")


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
    assert_close("gradient", g2.cpu().numpy(), g_ref, 1e-4)
    assert max(_loss_rel(s2.cpu().numpy(), s_ref)) < 1e-4
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
    if dtype == "bf16":
        ref["form"] = policy.act(OP.unpack(net, flat), net, obs, goal, prev, mask, h, c, u, quant="bf16")
        ref["form"]["u"] = u
    check_act(out2, ref, dtype, B, "autotuned")


@pytest.mark.parametrize("name,net,dtype,B", [("tiny", TINY_NET, "f32", 3), ("mini_resnet", MINI_RESNET, "bf16", 5),
                                              ("paper", C1.net, "f32", 4), ("paper", C1.net, "bf16", 4),
                                              ("mini_seresnext", MINI_SERESNEXT, "bf16", 3),
                                              ("seresnext_paper", SERESNEXT_NET, "f32", 4)])
def test_act_fused_forms_are_bit_identical(P, monkeypatch, name, net, dtype, B):
    """The act step's convolutions store their outputs (or split-K partials)
    group-major for the GroupNorm that reads them, and the stem's GroupNorm
    pools its own slab: the same values in another place and the same
    window maxima, so every act output equals the plain forms' bit for bit
    (tuned tiles, so that split-K partials are exercised)."""
    say(f"act fused forms {name} {dtype}")
    flat = R.init_params(net, 31, random_affine=True)
    g = np.random.default_rng(32)
    obs = g.random((B, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32)
    if dtype == "bf16":
        obs = R.round_bf16(obs)
    gw = {"raw": 2, "polar": 2}[net.goal_mode]
    goal = g.standard_normal((B, gw)).astype(np.float32)
    prev = g.integers(0, net.num_actions, B).astype(np.int32)
    mask = (g.random(B) > 0.3).astype(np.float32)
    h = (0.5 * g.standard_normal((net.lstm_layers, B, net.hidden))).astype(np.float32)
    c = (0.5 * g.standard_normal((net.lstm_layers, B, net.hidden))).astype(np.float32)
    u = g.random(B).astype(np.float32)
    n = P.Net(net, dtype)
    params = torch.tensor(flat, device=DEV)
    lp = P.cast_bf16(params) if dtype == "bf16" else None
    td = lambda a: torch.tensor(a, device=DEV)
    o = td(obs).to(torch.bfloat16) if dtype == "bf16" else td(obs)
    args = (o, td(goal), td(prev), td(mask), td(h), td(c), td(u), params, lp)
    n.autotune(1)
    gm = n.act(*args, want_logits=True)
    n.autotune(0)
    gm = {k: v.clone() for k, v in gm.items()}
    monkeypatch.setenv("DDPPO_ACT_FUSED", "0")
    plain = n.act(*args, want_logits=True)
    torch.cuda.synchronize()
    for k in ("logits", "value", "logp", "h", "c", "action"):
        assert torch.equal(gm[k], plain[k]), k


@pytest.mark.parametrize("net,dtype", [(RESNET_64, "f32"), (RESNET_64, "bf16"), (MINI_RESNET, "bf16")],
                         ids=["resnet64-f32", "resnet64-bf16", "mini_resnet-bf16"])
def test_learner_group_major_partials_are_bit_identical(P, monkeypatch, net, dtype):
    """In the learner the one-launch GroupNorms read their split-K partials
    group-major (the summed convolution output the backward needs is still
    stored plainly): loss statistics and the whole gradient equal the plain
    layout's bit for bit (tuned tiles)."""
    say(f"learner group-major partials {dtype}")
    T, N, envs, lengths = 3, 3, [2, 1, 0], [3, 2, 3]
    flat = R.init_params(net, 47, random_affine=True)
    rec = random_record(net, T, N, 48, lengths=lengths, bf16=dtype == "bf16")
    envs = sorted(envs, key=lambda e: -lengths[e])
    n = P.Net(net, dtype)
    params = torch.tensor(flat, device=DEV)
    lp = P.cast_bf16(params) if dtype == "bf16" else None
    ro = to_device(rec, bf16=dtype == "bf16")
    scale = torch.tensor([1.0], device=DEV)
    n.autotune(1)
    n.loss_backward(ro, envs, rec["lengths"], params, lp, P.LossCfg(), loss_scale=scale)
    n.autotune(0)
    g0, s0 = n.loss_backward(ro, envs, rec["lengths"], params, lp, P.LossCfg(), loss_scale=scale)
    g0, s0 = g0.clone(), s0.clone()
    monkeypatch.setenv("DDPPO_ACT_FUSED", "0")
    g1, s1 = n.loss_backward(ro, envs, rec["lengths"], params, lp, P.LossCfg(), loss_scale=scale)
    torch.cuda.synchronize()
    assert torch.equal(g0, g1) and torch.equal(s0, s1)


TILE_NAMES = ["128x128", "128x64", "64x128", "64x64", "128x32", "32x128"]


def test_every_tile_shape_on_the_act_products(P):
    """Every GEMM tile shape the autotuner may choose forced onto every
    product of a bfloat16 act step of the paper network (the tuned K split
    kept, and a split of 1): each within the tolerance of the oracle."""
    say("every tile shape on the act products (bf16, paper net)")
    net, B = C1.net, 4
    flat = R.init_params(net, 29, random_affine=True)
    g = np.random.default_rng(30)
    obs = R.round_bf16(g.random((B, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32))
    goal = g.standard_normal((B, 2)).astype(np.float32)
    prev = g.integers(0, net.num_actions, B).astype(np.int32)
    mask = np.ones(B, np.float32)
    h = (0.5 * g.standard_normal((net.lstm_layers, B, net.hidden))).astype(np.float32)
    c = (0.5 * g.standard_normal((net.lstm_layers, B, net.hidden))).astype(np.float32)
    u = g.random(B).astype(np.float32)
    n = P.Net(net, "bf16")
    params = torch.tensor(flat, device=DEV)
    lp = P.cast_bf16(params)
    td = lambda a: torch.tensor(a, device=DEV)
    args = (td(obs).to(torch.bfloat16), td(goal), td(prev), td(mask), td(h), td(c), td(u), params, lp)
    n.autotune(1)
    n.act(*args, want_logits=True)
    n.autotune(0)
    tuned = n.tile_table()
    assert tuned and all(r[5] < len(TILE_NAMES) for r in tuned)
    ref = policy.act(OP.unpack(net, flat), net, obs, goal, prev, mask, h, c, u)
    ref["u"] = u
    ref["form"] = policy.act(OP.unpack(net, flat), net, obs, goal, prev, mask, h, c, u, quant="bf16")
    ref["form"]["u"] = u
    for tile in range(len(TILE_NAMES)):
        for one_split in (False, True):
            n.tile_table([r[:5] + [tile, 1 if one_split else r[6]] for r in tuned])
            out = n.act(*args, want_logits=True)
            torch.cuda.synchronize()
            check_act(out, ref, "bf16", B, f"tile {TILE_NAMES[tile]}{' split 1' if one_split else ''}")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_stem_weight_gradient_tiles(P, dtype):
    """The channel-vector weight gradient (the stem's 4-channel input, k-pair
    LDS stores) forced onto every tile shape, with the tuned K split and with
    none: the whole gradient equals the tuned run's up to float32
    accumulation order."""
    say(f"stem weight-gradient tiles {dtype}")
    net, T, N, envs, lengths = RESNET_64, 3, 3, [2, 1, 0], [3, 2, 3]
    assert net.in_ch % 8 != 0 and net.in_ch % 4 == 0 and net.base_width % 8 == 0
    flat = R.init_params(net, 45, random_affine=True)
    rec = random_record(net, T, N, 46, lengths=lengths, bf16=dtype == "bf16")
    envs = sorted(envs, key=lambda e: -lengths[e])
    n = P.Net(net, dtype)
    params = torch.tensor(flat, device=DEV)
    lp = P.cast_bf16(params) if dtype == "bf16" else None
    ro = to_device(rec, bf16=dtype == "bf16")
    scale = torch.tensor([1.0], device=DEV)
    n.autotune(1)
    g0, _ = n.loss_backward(ro, envs, rec["lengths"], params, lp, P.LossCfg(), loss_scale=scale)
    n.autotune(0)
    g0 = g0.cpu().numpy().astype(np.float64)
    tuned = n.tile_table()
    rt = [r for r in tuned if r[0] == 4]          # the channel-vector weight-gradient problems
    assert rt, "no channel-vector weight gradient in the table"
    for tile in range(len(TILE_NAMES)):
        for split in (None, 1):
            n.tile_table([r[:5] + [tile, split or r[6]] for r in rt])
            g1, _ = n.loss_backward(ro, envs, rec["lengths"], params, lp, P.LossCfg(), loss_scale=scale)
            torch.cuda.synchronize()
            assert_close(f"gradient, tile {TILE_NAMES[tile]} split {split or 'tuned'}", g1.cpu().numpy(), g0, 1e-5)
