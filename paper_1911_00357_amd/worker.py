"""One DD-PPO worker on one GPU: collect a rollout with T+1 dependent act
steps, then GAE and E epochs x M minibatches of (loss backward, Adam).

Host-side sequencing only; every numeric step is a library call.  On one GPU
the gradient all-reduce between ppo_loss_backward and ppo_adam_step
(Eq. 3-4) is the identity.

Ragged rollouts (preempted envs, Sec. 3): envs must be ordered by length,
longest first, so the envs still collecting at step t are rows [0, B_t).
Env n is active at act steps t <= T_n; step T_n only supplies the bootstrap
value, and the next rollout starts from the state that step read.  A worker
preempted by the shared finished count (PreemptionMonitor) stops all its envs
at the same step T_w.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .api import Adam, LossCfg, Net, cast_bf16, gae


@dataclass
class PPOHyper:
    gamma: float = 0.99
    lam: float = 0.95
    clip: float = 0.2
    value_coef: float = 0.5
    entropy_coef: float = 0.01
    lr: float = 2.5e-4
    epochs: int = 2
    minibatches: int = 2
    norm_adv: bool = False


class Worker:
    def __init__(self, spec, dtype: str, T: int, N: int, params, hyper: PPOHyper = None, device="cuda", net=None):
        """net: an existing Net of this spec and dtype to share (its tile table
        and workspaces), else a new one."""
        self.hp = hyper or PPOHyper()
        self.spec, self.T, self.N, self.dev = spec, T, N, torch.device(device)
        self.net = net if net is not None else Net(spec, dtype)
        self.bf16 = dtype == "bf16"
        self.params = torch.as_tensor(np.asarray(params, np.float32)).to(self.dev).contiguous()
        assert self.params.numel() == self.net.P
        self.lp = cast_bf16(self.params) if self.bf16 else None
        self.adam = Adam(self.net.P, self.dev, lr=self.hp.lr,
                         loss_scale=65536.0 if self.bf16 else 1.0,
                         growth_interval=2000 if self.bf16 else 0)
        L, H, dev = spec.lstm_layers, spec.hidden, self.dev
        f32 = dict(dtype=torch.float32, device=dev)
        self.h_hist = torch.zeros(T + 1, L, N, H, **f32)    # state read by act step t
        self.c_hist = torch.zeros(T + 1, L, N, H, **f32)
        self.act_rec = torch.zeros(T + 2, N, dtype=torch.int32, device=dev)  # row 0: previous action
        self.logp = torch.zeros(T + 1, N, **f32)
        self.value = torch.zeros(T + 1, N, **f32)
        self.grad = torch.zeros(self.net.P, **f32)
        self.stats = torch.zeros(8, **f32)
        self.adv_stats = torch.zeros(2, dtype=torch.float64, device=dev)
        self.h_scr = torch.zeros(L, N, H, **f32)
        self.c_scr = torch.zeros(L, N, H, **f32)
        self.d_active = torch.full((T + 1,), N, dtype=torch.int32, device=dev)  # rows written per act step
        self._own_net = net is None

    def release(self):
        """Drop the library state now (before the interpreter's teardown),
        after the device has finished with it: the act graphs kept for this
        worker's buffers (all of a net it created; a shared net's owner clears
        its own) and the handles."""
        torch.cuda.synchronize()
        if self.net is not None and self._own_net:
            self.net.clear_graphs()
        self.net = None
        self.adam = None

    # ------------------------------------------------------------- rollout
    def collect(self, env: dict, lengths=None, graph: bool = False, trim: bool = False, monitor=None,
                iteration: int = 0):
        """env: device tensors obs [T+1,N,C,H,W], goal [T+1,N,2], mask [T+1,N],
        u [T+1,N].  lengths: host ints [N] (non-increasing) or None (all T).

        The T+1 act steps run in the library (ppo_collect).  Act step t writes
        the rows of the envs still collecting (T_n >= t) through a device row
        count (set from `lengths` before the steps run), so with graph=True one
        library-owned graph of the T+1 steps serves any lengths: the first call
        runs them eagerly and captures them, later calls launch the graph.
        trim=True instead launches step t on its active rows only (less
        computed, a graph per set of lengths).

        monitor: a PreemptionMonitor (Sec. 3).  The steps then run one at a
        time (with graph=True each launches its own captured graph), each
        waited for, and after each the monitor decides whether this worker's
        rollout ends there; the next step supplies the bootstrap value.
        Returns the rollout length T_w (None without a monitor)."""
        if monitor is not None:
            return self._collect_preemptible(env, graph, monitor, iteration)
        if not trim:
            self._set_active(lengths)
        self.net.collect(self._rollout_io(env), self.params, self.lp, active=None if trim else self.d_active,
                         lengths=lengths, trim=trim, graph=graph)
        return None

    def _rollout_io(self, env):
        return {"obs": env["obs"], "goal": env.get("goal"), "mask": env["mask"], "u": env["u"],
                "actions": self.act_rec, "logp": self.logp, "value": self.value, "h_hist": self.h_hist,
                "c_hist": self.c_hist, "h_last": self.h_scr, "c_last": self.c_scr}

    def _set_active(self, lengths):
        """Rows written at each act step: #{n : T_n >= t}, t = 0..T."""
        T, N = self.T, self.N
        lens = np.full(N, T) if lengths is None else np.asarray(lengths)
        assert lens.shape == (N,) and np.all(np.diff(lens) <= 0), "envs must be ordered longest first"
        counts = (lens[None, :] >= np.arange(T + 1)[:, None]).sum(axis=1).astype(np.int32)
        self.d_active.copy_(torch.from_numpy(counts))

    def _collect_preemptible(self, env, graph, monitor, iteration):
        from .preempt import collect as run_steps
        stream = torch.cuda.current_stream(self.dev)
        io = self._rollout_io(env)

        def step(t):
            self.net.collect(io, self.params, self.lp, steps=(t, t + 1), graph=graph)
            stream.synchronize()     # the monitor counts steps the device has finished

        Tw = run_steps(monitor, iteration, step)
        step(Tw)                     # the bootstrap step of every env
        return Tw

    def next_rollout_state(self, lengths=None):
        """Start state, previous action for the next rollout (env n resumes
        from the state its bootstrap step read)."""
        T, N = self.T, self.N
        lens = torch.as_tensor(np.full(N, T) if lengths is None else np.asarray(lengths),
                               dtype=torch.int64, device=self.dev)
        idx = torch.arange(N, device=self.dev)
        h0 = self.h_hist[lens, :, idx].permute(1, 0, 2).contiguous()
        c0 = self.c_hist[lens, :, idx].permute(1, 0, 2).contiguous()
        prev = self.act_rec[lens, idx].contiguous()
        return h0, c0, prev

    def start(self, h0, c0, prev_action):
        self.h_hist[0].copy_(h0)
        self.c_hist[0].copy_(c0)
        self.act_rec[0].copy_(prev_action)

    # -------------------------------------------------------------- update
    def rollout_view(self, env, adv, ret):
        return {"obs": env["obs"], "goal": env["goal"], "mask": env["mask"],
                "prev_action": self.act_rec[:-1], "action": self.act_rec[1:], "logp": self.logp,
                "adv": adv, "ret": ret, "h0": self.h_hist[0], "c0": self.c_hist[0]}

    def advantages(self, env, lengths=None):
        lens_dev = None if lengths is None else torch.as_tensor(np.asarray(lengths, np.int32),
                                                                device=self.dev)
        return gae(env["reward"], self.value, env["done"], lens_dev, self.hp.gamma, self.hp.lam,
                   stats=self.adv_stats)

    def update(self, env, partitions, lengths=None, on_minibatch=None):
        """GAE then, per epoch and minibatch, loss backward + Adam.
        partitions: per epoch a list of env-id arrays."""
        adv, ret = self.advantages(env, lengths)
        ro = self.rollout_view(env, adv, ret)
        cfg = LossCfg(self.hp.clip, self.hp.value_coef, self.hp.entropy_coef, self.hp.norm_adv)
        scale = self.adam.scale_tensor() if self.bf16 else None
        for ep in partitions:
            for envs in ep:
                self.net.loss_backward(ro, [int(e) for e in envs], lengths, self.params, self.lp, cfg,
                                       loss_scale=scale, adv_stats=self.adv_stats, grad=self.grad,
                                       stats=self.stats)
                if on_minibatch is not None:
                    on_minibatch(self)
                self.adam.step(self.params, self.grad, self.lp)
        return adv, ret

    def update_autograd(self, env, partitions, lengths=None):
        """The same update with the gradient taken through torch.autograd: the
        policy is a torch.autograd.Function whose backward recomputes the
        encoder and LSTM activations, and the PPO objective another whose
        forward and backward are ppo_loss_head (weights, loss scale and
        advantage normalisation applied in the library)."""
        from .autograd import policy, ppo_loss
        adv, ret = self.advantages(env, lengths)
        ro = self.rollout_view(env, adv, ret)
        cfg = LossCfg(self.hp.clip, self.hp.value_coef, self.hp.entropy_coef, self.hp.norm_adv)
        theta = self.params.detach().requires_grad_(True)   # shares storage with the master weights
        scale = self.adam.scale_tensor() if self.bf16 else None
        for ep in partitions:
            for envs in ep:
                envs = [int(e) for e in envs]
                logits, values, _ = policy(theta, self.net, ro, envs, lengths, self.lp)
                loss, self.stats = ppo_loss(logits, values, self.net, ro, envs, lengths, cfg, scale,
                                            self.adv_stats)
                (g,) = torch.autograd.grad(loss, theta)
                self.adam.step(self.params, g, self.lp)
        return adv, ret
