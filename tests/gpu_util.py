"""Shared helpers of the GPU parity tests: seeded rollout records in the
library's layout, the matching oracle minibatch, and per-tensor errors."""
import numpy as np
import torch

from synth import rollout as R
from synth.layout import tensor_list

DEV = "cuda"


def rel_err(x, ref, floor=1e-30):
    x, ref = np.asarray(x, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), floor))


def per_tensor_errors(net, g, g_ref):
    """{tensor name: relative L2 error} over the flat layout."""
    out = {}
    for t in tensor_list(net):
        n = int(np.prod(t.shape))
        sl = slice(t.offset, t.offset + n)
        out[t.name] = rel_err(g[sl], g_ref[sl], floor=1e-12)
    return out


def random_record(net, T, N, seed, lengths=None, bf16=False, logp_spread=0.3):
    """A synthetic rollout record [T+1][N] (act-step arrays) / [T][N]
    (transition arrays).  Old log-probs are random so both clip branches of
    the surrogate occur."""
    g = np.random.default_rng(seed)
    obs = g.random((T + 1, N, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32)
    if bf16:
        obs = R.round_bf16(obs)
    act = g.integers(0, net.num_actions, (T + 2, N)).astype(np.int32)
    return {
        "obs": obs,
        "goal": g.standard_normal((T + 1, N, 2)).astype(np.float32),
        "mask": (g.random((T + 1, N)) > 0.15).astype(np.float32),
        "act_rec": act,
        "logp": (np.log(0.25) + logp_spread * g.standard_normal((T + 1, N))).astype(np.float32),
        "adv": g.standard_normal((T, N)).astype(np.float32),
        "ret": g.standard_normal((T, N)).astype(np.float32),
        "h0": (0.5 * g.standard_normal((net.lstm_layers, N, net.hidden))).astype(np.float32),
        "c0": (0.5 * g.standard_normal((net.lstm_layers, N, net.hidden))).astype(np.float32),
        "lengths": np.full(N, T, np.int32) if lengths is None else np.asarray(lengths, np.int32),
    }


def to_device(rec, bf16=False):
    t = lambda a, dt=None: torch.as_tensor(np.ascontiguousarray(a)).to(DEV) if dt is None else \
        torch.as_tensor(np.ascontiguousarray(a)).to(DEV).to(dt)
    act = t(rec["act_rec"])
    return {
        "obs": t(rec["obs"], torch.bfloat16 if bf16 else torch.float32),
        "goal": t(rec["goal"]), "mask": t(rec["mask"]),
        "prev_action": act[:-1], "action": act[1:], "logp": t(rec["logp"]),
        "adv": t(rec["adv"]), "ret": t(rec["ret"]), "h0": t(rec["h0"]), "c0": t(rec["c0"]),
    }


def oracle_minibatch(rec, envs):
    """The oracle's minibatch dict for env set `envs` (time-major [T_B, B])."""
    envs = np.asarray(envs)
    lens = rec["lengths"][envs]
    TB = int(lens.max())
    a = rec["act_rec"]
    return {
        "envs": envs, "lens": lens,
        "obs": rec["obs"][:TB][:, envs].astype(np.float64),
        "goal": rec["goal"][:TB][:, envs].astype(np.float64),
        "prev_action": a[:TB][:, envs], "mask": rec["mask"][:TB][:, envs].astype(np.float64),
        "action": a[1:TB + 1][:, envs], "logp_old": rec["logp"][:TB][:, envs].astype(np.float64),
        "adv": rec["adv"][:TB][:, envs].astype(np.float64),
        "ret": rec["ret"][:TB][:, envs].astype(np.float64),
        "h0": rec["h0"][:, envs].astype(np.float64), "c0": rec["c0"][:, envs].astype(np.float64),
    }
