"""The persistent recurrence kernels (one launch per layer and direction, or
one launch for both layers of a 2-layer core pipelined a step apart, all time
steps) against the per-step kernels and the oracle, on packed ragged
minibatches."""
import os

import numpy as np
import pytest
import torch

from oracle import ppo
from synth import rollout as R
from synth.configs import TINY_NET, NetDesc, PPOCfg
from tests.gpu_util import DEV, oracle_minibatch, random_record, rel_err, to_device
from tests.nets import TINY_BIGCORE, TINY_CORE1024
from tests.test_gpu_parity import say

pytestmark = pytest.mark.gpu


# 2-layer core with 64 units: four units per workgroup in the recurrence kernels
TINY_2L64 = NetDesc(in_hw=32, avgpool=False, trunk="tiny", gn_groups=8, vis_hidden=64, goal_mode="polar",
                    goal_dim=8, prev_act_dim=8, lstm_layers=2, hidden=64)

# recurrence forms: both layers in one launch, one launch per layer, per-step kernels
MODES = {"seq2": ("1", "1"), "seq": ("1", "0"), "step": ("0", "0")}


def _run(P, net, dtype, T, N, envs, lengths, seed, mode):
    flat = R.init_params(net, seed, random_affine=True)
    rec = random_record(net, T, N, seed + 1, lengths=lengths, bf16=dtype == "bf16")
    envs = sorted(envs, key=lambda e: -rec["lengths"][e])
    n = P.Net(net, dtype)
    params = torch.tensor(flat, device=DEV)
    lp = P.cast_bf16(params) if dtype == "bf16" else None
    ro = to_device(rec, bf16=dtype == "bf16")
    names = ("DDPPO_LSTM_SEQ", "DDPPO_LSTM_SEQ2")
    old = {k: os.environ.get(k) for k in names}
    for k, v in zip(names, MODES[mode]):
        os.environ[k] = v
    try:
        grad, stats = n.loss_backward(ro, envs, rec["lengths"] if lengths is not None else None, params, lp,
                                      P.LossCfg(), loss_scale=torch.tensor([1.0], device=DEV))
        torch.cuda.synchronize()
    finally:
        for k in names:
            if old[k] is None:
                del os.environ[k]
            else:
                os.environ[k] = old[k]
    return flat, rec, envs, grad.cpu().numpy(), stats.cpu().numpy()


CASES = [
    ("bigcore", TINY_BIGCORE, 12, 5, [4, 0, 2, 1], [12, 3, 9, 7, 12]),
    ("bigcore_equal", TINY_BIGCORE, 8, 3, [0, 1, 2], None),
    ("tiny", TINY_NET, 16, 4, [0, 1, 2, 3], [16, 1, 11, 5]),
    ("tiny_2l64", TINY_2L64, 10, 6, [5, 0, 3, 1, 2], [10, 2, 7, 1, 10, 4]),
    ("core1024", TINY_CORE1024, 6, 3, [2, 0, 1], [6, 2, 5]),
]
TWO_LAYER = [c for c in CASES if c[1].lstm_layers == 2]


@pytest.mark.parametrize("name,net,T,N,envs,lengths", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_seq_matches_step_kernels(P, name, net, T, N, envs, lengths, dtype):
    say(f"lstm seq vs step {name} {dtype}")
    _, _, _, g_seq, s_seq = _run(P, net, dtype, T, N, envs, lengths, 11, "seq")
    _, _, _, g_step, s_step = _run(P, net, dtype, T, N, envs, lengths, 11, "step")
    assert np.all(np.isfinite(g_seq))
    # different summation orders: the persistent path really ran
    assert not np.array_equal(g_seq, g_step)
    tol = 1e-5 if dtype == "f32" else 2e-3
    e = rel_err(g_seq, g_step)
    say(f"  grad rel diff {e:.2e}; loss {s_seq[0]:.7f} vs {s_step[0]:.7f}")
    assert e < tol
    assert abs(s_seq[0] - s_step[0]) <= tol * max(abs(s_step[0]), 1e-6)


@pytest.mark.parametrize("name,net,T,N,envs,lengths", TWO_LAYER, ids=[c[0] for c in TWO_LAYER])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_seq2_matches_per_layer_and_step(P, name, net, T, N, envs, lengths, dtype):
    say(f"lstm seq2 vs seq / step {name} {dtype}")
    _, _, _, g2, s2 = _run(P, net, dtype, T, N, envs, lengths, 13, "seq2")
    _, _, _, g1, s1 = _run(P, net, dtype, T, N, envs, lengths, 13, "seq")
    _, _, _, g0, s0 = _run(P, net, dtype, T, N, envs, lengths, 13, "step")
    assert np.all(np.isfinite(g2))
    # the two-layer launch really ran (layer 0's input gradient is summed in another order)
    assert not np.array_equal(g2, g1)
    tol = 1e-5 if dtype == "f32" else 4e-3
    for g_ref, s_ref, what in ((g1, s1, "seq"), (g0, s0, "step")):
        e = rel_err(g2, g_ref)
        say(f"  vs {what}: grad rel diff {e:.2e}; loss {s2[0]:.7f} vs {s_ref[0]:.7f}")
        assert e < tol
        assert abs(s2[0] - s_ref[0]) <= tol * max(abs(s_ref[0]), 1e-6)


@pytest.mark.parametrize("core", ["512", "1024"])
@pytest.mark.parametrize("mode", ["seq2", "seq"])
@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("bf16", 2e-2)])
def test_seq_bigcore_vs_oracle(P, dtype, tol, mode, core):
    say(f"lstm {mode} vs oracle core {core} {dtype}")
    net = TINY_BIGCORE if core == "512" else TINY_CORE1024
    T, N, envs, lengths = 7, 4, [3, 1, 0], [7, 6, 2, 5]
    flat, rec, envs, g, s = _run(P, net, dtype, T, N, envs, lengths, 21, mode)
    mb = oracle_minibatch(rec, envs)
    s_ref, g_ref = ppo.loss_grad(flat.astype(np.float64), net, PPOCfg(), mb)
    e = rel_err(g, g_ref)
    say(f"  grad rel err {e:.2e}; loss {s[0]:.7f} vs {s_ref[0]:.7f}")
    assert e < tol
    denom = abs(s_ref[1]) + 0.5 * abs(s_ref[2]) + 0.01 * abs(s_ref[3])
    assert abs(s[0] - s_ref[0]) / denom < tol
