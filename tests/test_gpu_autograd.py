"""The policy behind torch.autograd.Function (hand-written backward with
recomputed encoder activations): against ppo_loss_backward, against the FP64
oracle on a 3-env x T=8 slice of the 128x128 differentiation workload, and
against finite differences of its own loss."""
import numpy as np
import pytest
import torch

from oracle import ppo
from synth import rollout as R
from synth.configs import C3, PPOCfg
from tests.gpu_util import DEV, assert_close, oracle_minibatch, random_record, rel_err, to_device
from tests.nets import TINY_PLUS
from tests.test_gpu_parity import LossCase, check_loss, gpu_decisions, oracle_refs, say

pytestmark = pytest.mark.gpu


def _setup(P, net, dtype, T, N, lengths, seed):
    flat = R.init_params(net, seed, random_affine=True)
    rec = random_record(net, T, N, seed + 1, lengths=lengths, bf16=dtype == "bf16")
    n = P.Net(net, dtype)
    params = torch.tensor(flat, device=DEV)
    lp = P.cast_bf16(params) if dtype == "bf16" else None
    return flat, rec, n, params, lp, to_device(rec, bf16=dtype == "bf16")


def _autograd_grad(P, n, ro, rec, envs, params, lp, N):
    """Gradient of the PPO loss through both autograd Functions (policy and
    ppo_loss_head), float32 (no loss scale)."""
    from paper_1911_00357_amd import autograd as AG
    th = params.clone().requires_grad_(True)
    logits, values, src = AG.policy(th, n, ro, envs, rec["lengths"], lp)
    loss, stats = AG.ppo_loss(logits, values, n, ro, envs, rec["lengths"])
    loss.backward()
    return th.grad.detach(), loss.detach(), stats, logits.detach(), values.detach()


@pytest.mark.parametrize("net,T,N,lengths,envs", [(TINY_PLUS, 6, 3, [6, 5, 3], [0, 1, 2]),
                                                  (C3.net, 8, 3, [8, 8, 8], [0, 1, 2])],
                         ids=["tiny+", "c3net"])
def test_autograd_matches_loss_backward(P, net, T, N, lengths, envs):
    say(f"autograd vs loss_backward {net.in_hw}")
    flat, rec, n, params, lp, ro = _setup(P, net, "f32", T, N, lengths, 31)
    g_ag, loss, st_ag, _, _ = _autograd_grad(P, n, ro, rec, envs, params, lp, N)
    g_lb, stats = n.loss_backward(ro, envs, rec["lengths"], params, lp)
    torch.cuda.synchronize()
    assert abs(loss.item() - stats[0].item()) <= 1e-5 * max(1.0, abs(stats[0].item()))
    assert_close("statistics", st_ag.cpu().numpy(), stats.cpu().numpy(), 1e-5)
    assert_close("gradient", g_ag.cpu().numpy(), g_lb.cpu().numpy(), 1e-5)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_autograd_c3_slice_vs_oracle(P, dtype):
    """3 envs x T=8 of the 128x128 network; the oracle takes the GPU's
    ReLU / max-pool decisions."""
    say(f"autograd c3 slice {dtype}")
    net = C3.net
    flat, rec, n, params, lp, ro = _setup(P, net, dtype, 8, 3, [8, 8, 8], 41)
    envs = [0, 1, 2]
    g, loss, stats, _, _ = _autograd_grad(P, n, ro, rec, envs, params, lp, 3)
    torch.cuda.synchronize()
    mb = oracle_minibatch(rec, envs)
    F = int(mb["lens"].sum())
    coded = gpu_decisions(n, net, F, len(envs), mb, codes=dtype == "bf16")
    dec = {k: v for k, v in coded.items() if not k.startswith("q:")}
    c = LossCase()
    c.g, c.s = g.cpu().numpy(), stats.cpu().numpy()
    oracle_refs(c, net, dtype, flat, mb, dec, coded=coded if dtype == "bf16" else None)
    check_loss(net, dtype, c, f"c3 slice {dtype}")


def test_autograd_c3_slice_finite_differences(P):
    """Central differences of the GPU's own FP32 loss along the gradient
    direction and along single-tensor random directions."""
    from paper_1911_00357_amd import autograd as AG
    net = C3.net
    flat, rec, n, params, lp, ro = _setup(P, net, "f32", 8, 3, [8, 8, 8], 43)
    envs = [0, 1, 2]
    g, loss, _, _, _ = _autograd_grad(P, n, ro, rec, envs, params, lp, 3)

    def L(th):
        with torch.no_grad():
            lg, v, _ = AG.policy(th, n, ro, envs, rec["lengths"], None)
            return AG.ppo_loss(lg, v, n, ro, envs, rec["lengths"])[0].double().item()

    names = {nm: (off, cnt) for nm, off, cnt in n.tensors()}
    rng = np.random.default_rng(0)
    dirs = [g / g.norm()]
    for nm in ("head.w", "lstm1.w", "fc.w", "enc.s3.b2.c3"):
        off, cnt = names[nm]
        d = torch.zeros_like(params)
        d[off:off + cnt] = torch.tensor(rng.standard_normal(cnt), dtype=torch.float32, device=DEV)
        dirs.append(d / d.norm())
    for d in dirs:
        gd = float((g.double() * d.double()).sum())
        h = 2e-3
        fd = (L(params + h * d) - L(params - h * d)) / (2 * h)
        say(f"  fd {fd:.6e} vs g.d {gd:.6e}")
        noise = 8 * 6e-8 * abs(float(loss)) / (2 * h)   # float32 rounding of the two losses
        assert abs(fd - gd) <= 2e-2 * abs(gd) + noise


@pytest.mark.parametrize("norm_adv", [False, True])
def test_worker_update_autograd_matches_update(P, norm_adv):
    """One update through torch.autograd moves the weights as the library's
    loss backward does (same Adam step on close gradients), with and without
    advantage normalisation."""
    from paper_1911_00357_amd.worker import PPOHyper, Worker
    say(f"worker update via autograd vs loss backward, norm_adv={norm_adv}")
    net, T, N = TINY_PLUS, 6, 3
    flat = R.init_params(net, 5, random_affine=True)
    g = np.random.default_rng(6)
    env = {"obs": torch.tensor(g.random((T + 1, N, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32), device=DEV),
           "goal": torch.tensor(g.standard_normal((T + 1, N, 2)).astype(np.float32), device=DEV),
           "mask": torch.tensor((g.random((T + 1, N)) > 0.1).astype(np.float32), device=DEV),
           "u": torch.tensor(g.random((T + 1, N)).astype(np.float32), device=DEV),
           "reward": torch.tensor(g.normal(0, 0.05, (T, N)).astype(np.float32), device=DEV),
           "done": torch.tensor((g.random((T, N)) < 0.1).astype(np.uint8), device=DEV)}
    lengths = [6, 5, 3]
    parts = [[np.array([0, 2]), np.array([1])]]
    deltas = []
    for ag in (False, True):
        w = Worker(net, "f32", T, N, flat, PPOHyper(norm_adv=norm_adv), device=DEV)
        w.collect(env, lengths)
        before = w.params.clone()
        (w.update_autograd if ag else w.update)(env, parts, lengths)
        torch.cuda.synchronize()
        deltas.append((w.params - before).cpu().numpy())
    e = rel_err(deltas[1], deltas[0])
    say(f"  weight-change rel diff {e:.2e}")
    assert np.abs(deltas[0]).max() > 0 and e < 1e-2
