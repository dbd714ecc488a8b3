"""The persistent recurrence kernels (one launch per layer and direction, all
time steps) against the per-step kernels and the oracle, on packed ragged
minibatches."""
import os

import numpy as np
import pytest
import torch

from oracle import ppo
from synth import rollout as R
from synth.configs import TINY_NET, PPOCfg
from tests.gpu_util import DEV, oracle_minibatch, random_record, rel_err, to_device
from tests.nets import TINY_BIGCORE
from tests.test_gpu_parity import say

pytestmark = pytest.mark.gpu


def _run(P, net, dtype, T, N, envs, lengths, seed, seq):
    flat = R.init_params(net, seed, random_affine=True)
    rec = random_record(net, T, N, seed + 1, lengths=lengths, bf16=dtype == "bf16")
    envs = sorted(envs, key=lambda e: -rec["lengths"][e])
    n = P.Net(net, dtype)
    params = torch.tensor(flat, device=DEV)
    lp = P.cast_bf16(params) if dtype == "bf16" else None
    ro = to_device(rec, bf16=dtype == "bf16")
    old = os.environ.get("DDPPO_LSTM_SEQ")
    os.environ["DDPPO_LSTM_SEQ"] = "1" if seq else "0"
    try:
        grad, stats = n.loss_backward(ro, envs, rec["lengths"] if lengths is not None else None, params, lp,
                                      P.LossCfg(), loss_scale=torch.tensor([1.0], device=DEV))
        torch.cuda.synchronize()
    finally:
        if old is None:
            del os.environ["DDPPO_LSTM_SEQ"]
        else:
            os.environ["DDPPO_LSTM_SEQ"] = old
    return flat, rec, envs, grad.cpu().numpy(), stats.cpu().numpy()


CASES = [
    ("bigcore", TINY_BIGCORE, 12, 5, [4, 0, 2, 1], [12, 3, 9, 7, 12]),
    ("bigcore_equal", TINY_BIGCORE, 8, 3, [0, 1, 2], None),
    ("tiny", TINY_NET, 16, 4, [0, 1, 2, 3], [16, 1, 11, 5]),
]


@pytest.mark.parametrize("name,net,T,N,envs,lengths", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_seq_matches_step_kernels(P, name, net, T, N, envs, lengths, dtype):
    say(f"lstm seq vs step {name} {dtype}")
    _, _, _, g_seq, s_seq = _run(P, net, dtype, T, N, envs, lengths, 11, True)
    _, _, _, g_step, s_step = _run(P, net, dtype, T, N, envs, lengths, 11, False)
    assert np.all(np.isfinite(g_seq))
    # different summation orders: the persistent path really ran
    assert not np.array_equal(g_seq, g_step)
    tol = 1e-5 if dtype == "f32" else 2e-3
    e = rel_err(g_seq, g_step)
    say(f"  grad rel diff {e:.2e}; loss {s_seq[0]:.7f} vs {s_step[0]:.7f}")
    assert e < tol
    assert abs(s_seq[0] - s_step[0]) <= tol * max(abs(s_step[0]), 1e-6)


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("bf16", 2e-2)])
def test_seq_bigcore_vs_oracle(P, dtype, tol):
    say(f"lstm seq vs oracle bigcore {dtype}")
    net, T, N, envs, lengths = TINY_BIGCORE, 7, 4, [3, 1, 0], [7, 6, 2, 5]
    flat, rec, envs, g, s = _run(P, net, dtype, T, N, envs, lengths, 21, True)
    mb = oracle_minibatch(rec, envs)
    s_ref, g_ref = ppo.loss_grad(flat.astype(np.float64), net, PPOCfg(), mb)
    e = rel_err(g, g_ref)
    say(f"  grad rel err {e:.2e}; loss {s[0]:.7f} vs {s_ref[0]:.7f}")
    assert e < tol
    denom = abs(s_ref[1]) + 0.5 * abs(s_ref[2]) + 0.01 * abs(s_ref[3])
    assert abs(s[0] - s_ref[0]) / denom < tol
