"""Seeded synthetic inputs standing in for Habitat renders of Gibson/MP3D.

The paper's frames come from a simulator and scene datasets that are not
available; these arrays have the same shapes and simple distributions:
  obs     ~ U[0,1)  [T+1, N, C, H, W]   (rounded to bfloat16 for BF16 workloads)
  goal    ~ N(0,1)  [T+1, N, 2]
  reward  = -0.01 + N(0, 0.05^2), done ~ Bernoulli(0.02), +2.5 where done   [T, N]
  u       ~ U[0,1)  [T+1, N]          uniforms for inverse-CDF action sampling
  lengths = T, or ~ U{T/4 .. T} for ragged workloads (the preemption floor
            of one quarter of the maximum rollout length, Sec. 3).
Random numbers the method draws (the sampling uniforms, the minibatch
permutation) are generated here and passed to both implementations.
The environment is action independent, so one rollout serves both sides.

This module holds none of the method's arithmetic.
"""
from __future__ import annotations

import numpy as np

from .configs import NetDesc, Workload
from .layout import tensor_list, param_count


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed, stream]))


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even float32 -> bfloat16 bit patterns (uint16)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    return r


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32)


def round_bf16(x: np.ndarray) -> np.ndarray:
    return bf16_bits_to_f32(to_bf16_bits(x))


def init_params(net: NetDesc, seed: int, random_affine: bool = False) -> np.ndarray:
    """FP32 flat parameter vector.  Convolutions Kaiming-uniform over the
    fan-in, fully connected and LSTM weights U(+-1/sqrt(fan_in)), biases 0,
    GroupNorm gamma 1 / beta 0, embedding N(0,1).  With random_affine the
    GroupNorm affine terms and all biases are drawn too (gradient tests)."""
    g = rng(seed, 1)
    p = np.zeros(param_count(net), dtype=np.float32)
    for t in tensor_list(net):
        n = int(np.prod(t.shape))
        sl = slice(t.offset, t.offset + n)
        if t.kind == "conv":
            b = np.sqrt(6.0 / t.fan_in)
            p[sl] = g.uniform(-b, b, n)
        elif t.kind == "fc":
            b = 1.0 / np.sqrt(t.fan_in)
            p[sl] = g.uniform(-b, b, n)
        elif t.kind == "emb":
            p[sl] = g.standard_normal(n)
        elif t.kind == "gn_g":
            p[sl] = g.uniform(0.5, 1.5, n) if random_affine else 1.0
        elif t.kind == "gn_b":
            p[sl] = g.uniform(-0.5, 0.5, n) if random_affine else 0.0
        elif t.kind == "bias":
            p[sl] = g.uniform(-0.2, 0.2, n) if random_affine else 0.0
    return p


def rollout_lengths(wl: Workload, seed: int) -> np.ndarray:
    if not wl.ragged:
        return np.full(wl.N, wl.T, dtype=np.int32)
    g = rng(seed, 2)
    return g.integers(wl.T // 4, wl.T + 1, size=wl.N).astype(np.int32)


def gen_obs(net: NetDesc, T1: int, N: int, seed: int, it: int, bf16: bool) -> np.ndarray:
    """Frames [T1, N, C, H, W] in float32 (bfloat16-representable if bf16)."""
    g = rng(seed, 100 + it)
    x = g.random((T1, N, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32)
    return round_bf16(x) if bf16 else x


def gen_rollout(wl: Workload, seed: int, it: int = 0, with_obs: bool = True) -> dict:
    """One iteration's environment stream."""
    T, N = wl.T, wl.N
    g = rng(seed, 200 + it)
    out = {}
    if with_obs:
        out["obs"] = gen_obs(wl.net, T + 1, N, seed, it, wl.dtype == "bf16")
    out["goal"] = g.standard_normal((T + 1, N, 2)).astype(np.float32)
    rew = (-0.01 + 0.05 * g.standard_normal((T, N))).astype(np.float32)
    done = (g.random((T, N)) < 0.02).astype(np.uint8)
    rew = (rew + 2.5 * done).astype(np.float32)
    out["reward"] = rew
    out["done"] = done
    out["u"] = g.random((T + 1, N)).astype(np.float32)
    out["lengths"] = rollout_lengths(wl, seed)
    # episode mask of each act step: 0 where an episode starts (the first
    # rollout, or the step after a done)
    mask = np.ones((T + 1, N), np.float32)
    mask[1:] = 1.0 - done
    if it == 0:
        mask[0] = 0.0
    else:
        prev = gen_rollout(wl, seed, it - 1, with_obs=False)
        last = prev["done"][prev["lengths"] - 1, np.arange(N)]
        mask[0] = 1.0 - last
    out["mask"] = mask
    return out


def gen_state(net: NetDesc, N: int, seed: int, zero: bool = True):
    """Recurrent state (h0, c0) [L, N, H] at the start of a rollout."""
    shape = (net.lstm_layers, N, net.hidden)
    if zero:
        return np.zeros(shape, np.float32), np.zeros(shape, np.float32)
    g = rng(seed, 3)
    return (0.5 * g.standard_normal(shape)).astype(np.float32), \
           (0.5 * g.standard_normal(shape)).astype(np.float32)


def partitions(wl: Workload, seed: int):
    """Per epoch, a seeded permutation of the envs split into equal minibatches
    (whole sequences per env)."""
    g = rng(seed, 4)
    parts = []
    for _ in range(wl.ppo.epochs):
        perm = g.permutation(wl.N).astype(np.int32)
        parts.append([np.sort(c) for c in np.array_split(perm, wl.ppo.minibatches)])
    return parts
