"""The paper-shaped worker at full size, in the configuration the benchmark
times: T = 128 act steps of N = 4 envs on 256x256 frames, replayed from one
captured graph, GEMM tiles autotuned in the warm-up (Sec. 4 "Training").
Checked on sampled outputs that the oracle computes one by one.

  act   a sampled step t is recomputed by the oracle from the GPU's own
        inputs of that step: frame, goal, previous action, mask, and the
        recurrent state the GPU carried into it.  Each sampled step is thus
        checked on its own, with no error carried over from earlier steps:
        value, the log-probability of the GPU's action, the next state, and
        the action (float32: identical; bfloat16: a different action only
        where u lies within the tolerance of a CDF step);
  GAE   over the whole rollout, from the GPU's values;
  loss  the first minibatch (2 envs x 128 steps = 256 frames, the rollout's
        own parameters) through the worker's update: the loss terms and
        every parameter tensor's gradient, the GPU's ReLU and max-pool
        decisions imposed and validated (float32).

bfloat16 act outputs on which the oracle's bfloat16 precision form, with
its own roundings, already reaches AT_RISK are reported, not held to the bar.
"""
import numpy as np
import pytest
import torch

from oracle import nn as onn
from oracle import params as OP
from oracle import policy, ppo
from synth import rollout as R
from synth.configs import C1, C2
from tests.gpu_util import assert_close, errs, flip_summary, tensor_errors
from tests.test_gpu_parity import (AT_RISK, TOL, LossCase, _loss_rel, assert_actions_agree, gpu_decisions,
                                   oracle_refs, say)
from tests.test_gpu_worker import _stage

pytestmark = pytest.mark.gpu
STEPS = (0, 1, 37, 64, 127, 128)


def _worker(wl, seed):
    import paper_1911_00357_amd as PP
    from paper_1911_00357_amd.worker import PPOHyper, Worker
    net = PP.Net(wl.net, wl.dtype)
    net.autotune(1)                    # tiles and K splits tuned on the first (eager) pass, as the benchmark does
    flat = R.init_params(wl.net, seed)
    p = wl.ppo
    hp = PPOHyper(p.gamma, p.lam, p.clip, p.value_coef, p.entropy_coef, p.lr, p.epochs, p.minibatches, p.norm_adv)
    w = Worker(wl.net, wl.dtype, wl.T, wl.N, flat, hp, "cuda", net=net)
    ro, env = _stage(wl, seed)
    w.collect(env, None, graph=True)   # eager pass (tuning), capture, replay
    net.autotune(0)
    w.collect(env, None, graph=True)   # the replay the benchmark times
    torch.cuda.synchronize()
    return w, flat, ro, env


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_full_size_act_loop_sampled_steps(P, dtype):
    wl = C1 if dtype == "f32" else C2
    net, T, N = wl.net, wl.T, wl.N
    say(f"full-size act loop {dtype}: T={T} N={N}, sampled steps {STEPS}")
    w, flat, ro, env = _worker(wl, seed=7)
    Po = OP.unpack(net, flat)
    tol = TOL[dtype]
    g = lambda x: x.cpu().numpy()
    h_hist, c_hist, act_rec = g(w.h_hist), g(w.c_hist), g(w.act_rec)
    value, logp = g(w.value), g(w.logp)
    for t in STEPS:
        h_in, c_in, prev = h_hist[t], c_hist[t], act_rec[t]
        args = (Po, net, ro["obs"][t], ro["goal"][t], prev, ro["mask"][t], h_in, c_in, ro["u"][t])
        ref = policy.act(*args)
        form = policy.act(*args, quant="bf16") if dtype == "bf16" else None
        h_out = g(w.h_scr) if t == T else h_hist[t + 1]
        c_out = g(w.c_scr) if t == T else c_hist[t + 1]
        a = act_rec[t + 1]
        lp_ref = onn.log_softmax(ref["logits"])[np.arange(N), a]
        outs = {"value": (value[t], ref["value"]), "logp": (logp[t], lp_ref), "h": (h_out, ref["h"]),
                "c": (c_out, ref["c"])}
        line = []
        for k, (x, r) in outs.items():
            e = errs(x, r)
            line.append(f"{k} {e[0]:.1e}/{e[1]:.1e}")
            if form is not None:
                rf = onn.log_softmax(form["logits"])[np.arange(N), a] if k == "logp" else form[k]
                ef = errs(rf, r)
                line[-1] += f" (form {ef[0]:.1e})"
                if max(ef) >= AT_RISK:
                    continue
            assert_close(f"step {t} {k}", x, r, tol)
        if dtype == "f32":
            np.testing.assert_array_equal(a, ref["action"])
        else:
            assert_actions_agree(a, {"action": ref["action"], "logits": ref["logits"], "u": ro["u"][t]}, tol)
        say(f"  step {t}: " + "; ".join(line) + f"; actions differing {int((a != ref['action']).sum())}")
    # GAE over the whole rollout from the GPU's values
    adv, ret = w.advantages(env)
    torch.cuda.synchronize()
    A, Rt = ppo.gae(ro["reward"], value, ro["done"], ro["lengths"], wl.ppo.gamma, wl.ppo.lam)
    assert_close("advantages", g(adv), A, 1e-5)
    assert_close("returns", g(ret), Rt, 1e-5)
    w.release()


def test_full_size_first_minibatch_f32(P):
    wl = C1
    net, T, N = wl.net, wl.T, wl.N
    say(f"full-size first minibatch f32: 2 envs x T={T}")
    w, flat, ro, env = _worker(wl, seed=9)
    g = lambda x: x.cpu().numpy()
    parts = R.partitions(wl, 9)
    envs0 = np.asarray(parts[0][0])
    rec = {"prev_action": g(w.act_rec[:-1]), "mask": ro["mask"], "action": g(w.act_rec[1:]), "logp": g(w.logp),
           "h0": g(w.h_hist[0]), "c0": g(w.c_hist[0])}
    # the update's own GAE (deterministic: the update recomputes the same values)
    adv_t, ret_t = w.advantages(env)
    adv_g, ret_g = g(adv_t), g(ret_t)
    hooked = {}

    def on_minibatch(wk):
        if hooked:
            return
        torch.cuda.synchronize()
        mb = ppo.minibatch_inputs(net, ro, rec, adv_g, ret_g, envs0)
        hooked.update(grad=g(wk.grad).astype(np.float64), stats=g(wk.stats).astype(np.float64), mb=mb,
                      dec=gpu_decisions(wk.net, net, int(mb["lens"].sum()), len(envs0), mb))

    w.update(env, parts, None, on_minibatch=on_minibatch)
    torch.cuda.synchronize()
    st = w.adam.state()
    assert st["skipped"] == 0 and not w.net.recurrence_failed()
    c = LossCase()
    c.g, c.s = hooked["grad"], hooked["stats"]
    oracle_refs(c, net, "f32", flat, hooked["mb"], hooked["dec"])
    tol = TOL["f32"]
    lerr = max(_loss_rel(c.s, c.s_exact))
    er = tensor_errors(net, c.g, c.g_exact)
    worst = sorted(er.items(), key=lambda kv: -max(kv[1]))[:4]
    say(f"  loss {c.s[0]:.6f} vs {c.s_exact[0]:.6f} ({lerr:.1e}); gradient {errs(c.g, c.g_exact)}; "
        f"ratio [{c.s[6]:.7f}, {c.s[7]:.7f}]; {flip_summary(c.flips)}; worst tensors "
        + ", ".join(f"{k}=({a:.1e},{b:.1e})" for k, (a, b) in worst))
    assert lerr < tol
    assert_close("gradient", c.g, c.g_exact, tol)
    assert all(max(v) < tol for v in er.values()), worst
    # the rollout's own parameters: every probability ratio is 1
    assert abs(c.s[6] - 1) < 1e-5 and abs(c.s[7] - 1) < 1e-5
    w.release()
