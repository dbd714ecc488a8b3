"""FP64 CPU oracle for the DD-PPO worker hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The HIP library
never calls it, and it shares no code with the library: it reads the flat
parameter format with its own code, computes every step in float64 with
numpy, and differentiates by hand.

Contents
  nn      convolution, GroupNorm, pooling, LSTM cell, log-softmax (fwd + bwd)
  policy  the agent of the paper's appendix "Agent Design": encoder, goal
          encoder, previous-action embedding, LSTM core, policy/value heads,
          inverse-CDF sampling; forward over sequences and hand backward
  ppo     GAE, advantage statistics, the clipped PPO loss (Eq. 2) with its
          gradient, Adam, and the worker update loop (Sec. 3-4)
  preempt the preemption threshold of Sec. 3: rollout length per worker from
          per-step durations
Parity status per function is stated in each module's header.
"""
from . import nn, params, policy, ppo, preempt  # noqa: F401
