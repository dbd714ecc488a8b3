"""Python binding of the C ABI (include/ddppo.h) over torch device tensors.

Argument marshalling only: every step of the path runs in the HIP kernels of
libddppo.so.  Tensors must be CUDA (HIP) tensors, contiguous, with the dtypes
the header states; work is enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

from . import _lib as L
from ._lib import check, lib


# Test aid: fill workspaces with NaN bytes before every call.
POISON_WS = os.environ.get("DDPPO_POISON_WS", "0") == "1"

_live_nets = [0]   # ppo_net handles not yet destroyed


def live_nets() -> int:
    """Library handles (ppo_net) alive now: 0 once every Net is gone, so that
    no library state (graphs, events, streams) outlives the caller's work."""
    return _live_nets[0]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, name, numel=None):
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements, got {t.numel()}")
    return t


def _stream(device=None):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def desc_from(spec, dtype: str) -> L.NetDesc:
    """Build the C description from any object with the network fields
    (in_ch, in_hw, avgpool, trunk 'tiny'|'resnet'|'seresnext', tiny_ch,
    base_width, blocks, gn_groups, compress_ch, vis_hidden, goal_mode
    'raw'|'polar', goal_dim, prev_act_dim, lstm_layers, hidden, num_actions,
    and for seresnext cardinality, se_reduction)."""
    d = L.NetDesc()
    d.in_ch, d.in_hw, d.avgpool = spec.in_ch, spec.in_hw, int(bool(spec.avgpool))
    trunks = {"tiny": L.PPO_TRUNK_TINY, "resnet": L.PPO_TRUNK_RESNET, "seresnext": L.PPO_TRUNK_SERESNEXT,
              "none": L.PPO_TRUNK_NONE}
    if spec.trunk not in trunks:
        raise ValueError(f"unknown trunk {spec.trunk!r}")
    d.trunk = trunks[spec.trunk]
    d.cardinality = getattr(spec, "cardinality", 0)
    d.se_reduction = getattr(spec, "se_reduction", 0)
    d.tiny_ch[0], d.tiny_ch[1] = spec.tiny_ch
    d.base_width = spec.base_width
    for i in range(4):
        d.blocks[i] = spec.blocks[i]
    d.gn_groups, d.compress_ch, d.vis_hidden = spec.gn_groups, spec.compress_ch, spec.vis_hidden
    goals = {"raw": L.PPO_GOAL_RAW, "polar": L.PPO_GOAL_POLAR, "vec3": L.PPO_GOAL_VEC3, "none": L.PPO_GOAL_NONE}
    if spec.goal_mode not in goals:
        raise ValueError(f"unknown goal mode {spec.goal_mode!r}")
    d.goal_mode = goals[spec.goal_mode]
    d.prev_actions = getattr(spec, "prev_actions", 0)
    d.goal_dim, d.prev_act_dim = spec.goal_dim, spec.prev_act_dim
    d.lstm_layers, d.hidden, d.num_actions = spec.lstm_layers, spec.hidden, spec.num_actions
    d.dtype = L.PPO_BF16 if dtype == "bf16" else L.PPO_F32
    return d


@dataclass
class LossCfg:
    clip: float = 0.2
    value_coef: float = 0.5
    entropy_coef: float = 0.01
    norm_adv: bool = False


class Net:
    """A ppo_net plus cached workspaces."""

    def __init__(self, spec, dtype: str = "f32"):
        self.spec = spec
        self.dtype = dtype
        self.bf16 = dtype == "bf16"
        d = desc_from(spec, dtype)
        h = C.c_void_p()
        check(lib().ppo_net_create(C.byref(d), C.byref(h)), "ppo_net_create")
        self._h = h
        _live_nets[0] += 1
        self.P = int(lib().ppo_param_count(h))
        self.L, self.H, self.A = spec.lstm_layers, spec.hidden, spec.num_actions
        self.flat = int(spec.flat_dim)      # width of the visual FC's input (the encoder's output)
        self._ws = {}
        self._last_learn = None   # (frames, envs) of the last learner call

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().ppo_net_destroy(h)
                _live_nets[0] -= 1
            except Exception:
                pass

    def tensors(self):
        out, i = [], 0
        while True:
            name, off, cnt = C.c_char_p(), C.c_size_t(), C.c_size_t()
            if lib().ppo_param_tensor(self._h, i, C.byref(name), C.byref(off), C.byref(cnt)) != 0:
                return out
            out.append((name.value.decode(), off.value, cnt.value))
            i += 1

    def workspace_bytes(self, op: int, max_frames: int, max_envs: int = 1) -> int:
        b = C.c_size_t()
        check(lib().ppo_workspace_size(self._h, op, max_frames, max_envs, C.byref(b)),
              "ppo_workspace_size")
        return b.value

    def workspace(self, op: int, max_frames: int, max_envs: int, device) -> torch.Tensor:
        need = self.workspace_bytes(op, max_frames, max_envs)
        key = (op, str(device))
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=device)
            self._ws[key] = ws
        if POISON_WS and not torch.cuda.is_current_stream_capturing():
            ws.fill_(0xFF)  # every byte 0xff: a float read of unwritten scratch is NaN
        return ws

    def probe(self, op: int, max_frames: int, max_envs: int, kind: int, index: int = 0):
        """Location of saved forward activations in a workspace (test aid):
        (name, relu, byte offset, dims)."""
        name, relu, off = C.c_char_p(), C.c_int(), C.c_size_t()
        dims = (C.c_int * 4)()
        check(lib().ppo_workspace_probe(self._h, op, max_frames, max_envs, kind, index, C.byref(name),
                                        C.byref(relu), C.byref(off), dims), "ppo_workspace_probe")
        return (name.value.decode() if name.value else ""), relu.value, off.value, list(dims)

    def bench_unit_gemm(self, op: int, unit: int, frames: int, params, params_lp, grad, reps: int):
        """Enqueue `reps` launches of one trunk unit's convolution GEMM (benchmark
        aid); returns the algorithmic FLOPs of one launch."""
        dev = params.device
        ws = self.workspace(L.PPO_OP_LEARN, frames, 1, dev)
        fl = C.c_double()
        check(lib().ppo_bench_unit_gemm(self._h, op, unit, frames, _ptr(params), _ptr(params_lp), _ptr(grad),
                                        _ptr(ws), ws.numel(), reps, C.byref(fl), _stream(dev)),
              "ppo_bench_unit_gemm")
        return fl.value

    def autotune(self, mode: int) -> int:
        """1: tune GEMM tiles of new problems in later calls (waits on the GPU);
        0: stop tuning, keep the table; -1: clear it.  Returns table entries."""
        n = C.c_int()
        check(lib().ppo_autotune(self._h, mode, C.byref(n)), "ppo_autotune")
        return n.value

    def tile_table(self, rows=None):
        """The autotuner's table as a list of 7-int rows (key, tile, split);
        with rows, load them into the table first."""
        n = C.c_int(0)
        if rows:
            buf = (C.c_int64 * (7 * len(rows)))(*[int(v) for r in rows for v in r])
            n.value = len(rows)
            check(lib().ppo_autotune_table(self._h, 1, buf, len(rows), C.byref(n)), "ppo_autotune_table")
        check(lib().ppo_autotune_table(self._h, 0, None, 0, C.byref(n)), "ppo_autotune_table")
        buf = (C.c_int64 * (7 * max(n.value, 1)))()
        cap = n.value
        check(lib().ppo_autotune_table(self._h, 0, buf, cap, C.byref(n)), "ppo_autotune_table")
        return [list(buf[7 * i:7 * i + 7]) for i in range(min(n.value, cap))]

    def gemm_timer_arm(self, unit: int, op: int, max_launches: int = 4096):
        """Time the GEMM kernel launches of one trunk unit (L.PPO_TIMER_ALL_UNITS:
        all) and op in later calls (benchmark aid; unit -1 disarms)."""
        check(lib().ppo_gemm_timer_arm(self._h, unit, op, max_launches), "ppo_gemm_timer_arm")

    def gemm_timer_read(self):
        """(launches, summed ms, summed 2*M*N*K, summed weight bytes) since the
        last read."""
        n, ms, fl, wb = C.c_int(), C.c_double(), C.c_double(), C.c_double()
        check(lib().ppo_gemm_timer_read(self._h, C.byref(n), C.byref(ms), C.byref(fl), C.byref(wb)),
              "ppo_gemm_timer_read")
        return n.value, ms.value, fl.value, wb.value

    def recurrence_failed(self) -> bool:
        """True if a persistent LSTM launch of the last learner call gave up
        at a barrier (its outputs are then NaN); synchronises the stream."""
        ws = self.last_workspace(L.PPO_OP_LEARN)
        if ws is None or self._last_learn is None:
            return False
        off = self.probe(L.PPO_OP_LEARN, *self._last_learn, 4)[2]
        return bool(ws[off:off + 4].view(torch.int32).item())

    def last_workspace(self, op: int):
        return self._ws.get((op, "cuda:0")) if self._ws else None

    # ------------------------------------------------------------------ act
    def act(self, obs, goal, prev_action, mask, h_in, c_in, u, params, params_lp=None,
            out=None, want_logits=False, state_rows=0, active=None):
        """One act step for B = obs.shape[0] envs.  h_in/c_in [L, state_rows, H]
        (state_rows = B by default); rows < B are read and written.  active: a
        one-element device int32 tensor; only rows < active[0] (read on the
        device) are written."""
        B = obs.shape[0]
        SR = state_rows or B
        odt = torch.bfloat16 if self.bf16 and self.spec.trunk != "none" else torch.float32
        _need(obs, odt, "obs")
        gw = {"raw": 2, "polar": 2, "vec3": 3}.get(self.spec.goal_mode, 0)
        if gw:
            _need(goal, torch.float32, "goal", B * gw)
        _need(mask, torch.float32, "mask", B)
        # rows < B of every layer are read: at least (L-1)*SR*H + B*H elements
        need_state = (self.L - 1) * SR * self.H + B * self.H
        for nm, t in (("h_in", h_in), ("c_in", c_in)):
            _need(t, torch.float32, nm)
            if t.numel() < need_state:
                raise ValueError(f"{nm} holds {t.numel()} elements, needs {need_state}")
        _need(u, torch.float32, "u", B)
        _need(params, torch.float32, "params", self.P)
        if self.spec.prev_act_dim:
            _need(prev_action, torch.int32, "prev_action", B)
        if self.bf16:
            _need(params_lp, torch.bfloat16, "params_lp", self.P)
        dev = obs.device
        if out is None:
            out = {"action": torch.empty(B, dtype=torch.int32, device=dev),
                   "logp": torch.empty(B, dtype=torch.float32, device=dev),
                   "value": torch.empty(B, dtype=torch.float32, device=dev),
                   "h": torch.empty_like(h_in), "c": torch.empty_like(c_in)}
            if want_logits:
                out["logits"] = torch.empty(B, self.A, dtype=torch.float32, device=dev)
        io = L.ActIO()
        io.batch = B
        io.state_rows = SR
        io.obs, io.goal, io.prev_action, io.mask = _ptr(obs), _ptr(goal), _ptr(prev_action), _ptr(mask)
        io.h_in, io.c_in, io.u = _ptr(h_in), _ptr(c_in), _ptr(u)
        io.params, io.params_lp = _ptr(params), _ptr(params_lp)
        io.action, io.logp, io.value = _ptr(out["action"]), _ptr(out["logp"]), _ptr(out["value"])
        for nm in ("h", "c"):
            _need(out[nm], torch.float32, "out." + nm)
            if out[nm].numel() < need_state:
                raise ValueError(f"out.{nm} holds {out[nm].numel()} elements, needs {need_state}")
        io.h_out, io.c_out = _ptr(out["h"]), _ptr(out["c"])
        io.logits = _ptr(out.get("logits"))
        if active is not None:
            _need(active, torch.int32, "active", 1)
        io.active = _ptr(active)
        ws = self.workspace(L.PPO_OP_ACT, B, 1, dev)
        check(lib().ppo_act(self._h, C.byref(io), _ptr(ws), ws.numel(), _stream(dev)), "ppo_act")
        return out

    def collect(self, ro, params, params_lp=None, steps=None, active=None, lengths=None, trim=False,
                graph=False):
        """The rollout's act steps through ppo_collect.  ro: device tensors
        'obs' [T+1, N, ...], 'goal' [T+1, N, gw] (or None), 'mask', 'u'
        [T+1, N], 'actions' [T+2, N] int32 (row 0 read), 'logp', 'value'
        [T+1, N], 'h_hist', 'c_hist' [T+1, L, N, H] (row 0 read), 'h_last',
        'c_last' [L, N, H].  steps: (t_begin, t_end), default all T+1.
        active: device int32 [T+1] row counts; lengths with trim=True: host
        T_n (non-increasing) for per-step batches.  graph=True: launch the
        library's captured graph of these arguments."""
        T1, N = ro["mask"].shape[0], ro["mask"].shape[1]
        T = T1 - 1
        odt = torch.bfloat16 if self.bf16 and self.spec.trunk != "none" else torch.float32
        _need(ro["obs"], odt, "obs")
        if ro["obs"].numel() != T1 * N * self.spec.in_ch * self.spec.in_hw * self.spec.in_hw:
            raise ValueError("obs must be [T+1, N, C, H, W]")
        gw = {"raw": 2, "polar": 2, "vec3": 3}.get(self.spec.goal_mode, 0)
        if gw:
            _need(ro["goal"], torch.float32, "goal", T1 * N * gw)
        for k in ("mask", "u", "logp", "value"):
            _need(ro[k], torch.float32, k, T1 * N)
        _need(ro["actions"], torch.int32, "actions", (T + 2) * N)
        state = self.L * N * self.H
        for k, n in (("h_hist", T1 * state), ("c_hist", T1 * state), ("h_last", state), ("c_last", state)):
            _need(ro[k], torch.float32, k, n)
        _need(params, torch.float32, "params", self.P)
        if self.bf16:
            _need(params_lp, torch.bfloat16, "params_lp", self.P)
        if active is not None:
            _need(active, torch.int32, "active", T1)
        t0, t1 = steps if steps is not None else (0, T1)
        io = L.CollectIO()
        io.T, io.N, io.t_begin, io.t_end = T, N, t0, t1
        io.obs, io.goal, io.mask, io.u = _ptr(ro["obs"]), _ptr(ro.get("goal")), _ptr(ro["mask"]), _ptr(ro["u"])
        io.active = _ptr(active)
        lens = None
        if trim and lengths is not None:
            lens = (C.c_int32 * N)(*[int(x) for x in lengths])
            io.lengths = C.cast(lens, L.P_i32)
        io.params, io.params_lp = _ptr(params), _ptr(params_lp)
        io.actions, io.logp, io.value = _ptr(ro["actions"]), _ptr(ro["logp"]), _ptr(ro["value"])
        io.h_hist, io.c_hist, io.h_last, io.c_last = (_ptr(ro[k]) for k in ("h_hist", "c_hist", "h_last", "c_last"))
        flags = (L.PPO_COLLECT_GRAPH if graph else 0) | (L.PPO_COLLECT_TRIM if trim else 0)
        dev = ro["obs"].device
        ws = self.workspace(L.PPO_OP_ACT, N, 1, dev)
        check(lib().ppo_collect(self._h, C.byref(io), flags, _ptr(ws), ws.numel(), _stream(dev)), "ppo_collect")

    def clear_graphs(self) -> int:
        """Drop the act graphs the library keeps for this net (waits for the device)."""
        return int(lib().ppo_collect_clear(self._h))

    def graph_count(self) -> int:
        """Act graphs the library keeps for this net."""
        return int(lib().ppo_collect_graph_count(self._h))

    # -------------------------------------------------------------- learner
    def _batch(self, ro, env_ids, lengths, params, params_lp, learner=True, inputs=True):
        """The ppo_batch of a minibatch.  learner: the loss fields (actions,
        old log-probs, advantages, returns); inputs: the policy inputs."""
        T1, N = ro["mask"].shape[0], ro["mask"].shape[1]
        T = T1 - 1
        fields = [("mask", torch.float32, T1 * N)]
        if inputs:
            # a features-in net reads float32 feature vectors in both precisions
            _need(ro["obs"], torch.bfloat16 if self.bf16 and self.spec.trunk != "none" else torch.float32, "obs")
            fields += [("h0", torch.float32, self.L * N * self.H), ("c0", torch.float32, self.L * N * self.H)]
            gw = {"raw": 2, "polar": 2, "vec3": 3}.get(self.spec.goal_mode, 0)
            if gw:
                fields.append(("goal", torch.float32, T1 * N * gw))
        if learner:
            fields += [("action", torch.int32, T1 * N), ("logp", torch.float32, T1 * N),
                       ("adv", torch.float32, T * N), ("ret", torch.float32, T * N)]
        for k, dt, n in fields:
            _need(ro[k], dt, k, n)
        if inputs:
            if self.spec.prev_act_dim:
                _need(ro["prev_action"], torch.int32, "prev_action", T1 * N)
            _need(params, torch.float32, "params", self.P)
            if self.bf16:
                _need(params_lp, torch.bfloat16, "params_lp", self.P)
        env = (C.c_int32 * len(env_ids))(*[int(e) for e in env_ids])
        lens = None
        F = T * len(env_ids)
        if lengths is not None:
            lens = (C.c_int32 * N)(*[int(x) for x in lengths])
            F = int(sum(int(lengths[int(e)]) for e in env_ids))
        b = L.Batch()
        b.T, b.N, b.nb = T, N, len(env_ids)
        b.env_ids = C.cast(env, L.P_i32)
        b.lengths = C.cast(lens, L.P_i32) if lens is not None else None
        b.mask = _ptr(ro["mask"])
        if inputs:
            b.obs, b.goal, b.prev_action = _ptr(ro["obs"]), _ptr(ro.get("goal")), _ptr(ro.get("prev_action"))
            b.h0, b.c0 = _ptr(ro["h0"]), _ptr(ro["c0"])
            b.params, b.params_lp = _ptr(params), _ptr(params_lp)
        if learner:
            b.action, b.logp_old, b.adv, b.ret = (_ptr(ro["action"]), _ptr(ro["logp"]),
                                                  _ptr(ro["adv"]), _ptr(ro["ret"]))
        return b, (env, lens), F, ro["mask"].device

    def loss_backward(self, ro: dict, env_ids, lengths, params, params_lp=None, cfg: LossCfg = None,
                      loss_scale=None, adv_stats=None, grad=None, stats=None):
        """ro: device rollout dict with obs [T+1,N,C,H,W], goal [T+1,N,2],
        prev_action/action [T+1,N] int32, mask/logp [T+1,N], adv/ret [T,N],
        h0/c0 [L,N,H].  env_ids: host ints; lengths: host ints [N] or None."""
        cfg = cfg or LossCfg()
        b, keep, F, dev = self._batch(ro, env_ids, lengths, params, params_lp)
        c = L.LossCfg()
        c.clip, c.value_coef, c.entropy_coef = cfg.clip, cfg.value_coef, cfg.entropy_coef
        c.norm_adv = int(cfg.norm_adv)
        c.adv_stats = _ptr(adv_stats)
        if grad is None:
            grad = torch.empty(self.P, dtype=torch.float32, device=dev)
        if stats is None:
            stats = torch.empty(8, dtype=torch.float32, device=dev)
        ws = self.workspace(L.PPO_OP_LEARN, F, len(env_ids), dev)
        self._last_learn = (F, len(env_ids))
        check(lib().ppo_loss_backward(self._h, C.byref(b), C.byref(c), _ptr(loss_scale), _ptr(grad),
                                      _ptr(stats), _ptr(ws), ws.numel(), _stream(dev)),
              "ppo_loss_backward")
        return grad, stats

    def policy_forward(self, ro, env_ids, lengths, params, params_lp=None):
        """logits [F, A], values [F], frame_src [F] (t*N + env) of every valid
        minibatch frame, in the library's packed order."""
        b, keep, F, dev = self._batch(ro, env_ids, lengths, params, params_lp, learner=False)
        logits = torch.empty(F, self.A, dtype=torch.float32, device=dev)
        values = torch.empty(F, dtype=torch.float32, device=dev)
        src = torch.empty(F, dtype=torch.int32, device=dev)
        ws = self.workspace(L.PPO_OP_LEARN, F, len(env_ids), dev)
        self._last_learn = (F, len(env_ids))
        check(lib().ppo_policy_forward(self._h, C.byref(b), _ptr(logits), _ptr(values), _ptr(src), _ptr(ws),
                                       ws.numel(), _stream(dev)), "ppo_policy_forward")
        return logits, values, src

    def loss_head(self, ro, env_ids, lengths, logits, values, cfg: LossCfg = None, loss_scale=None,
                  adv_stats=None, dlogits=None, dvalues=None, stats=None, loss_out=None):
        """The PPO objective on given policy outputs (frames in policy_forward's
        order): (dlogits [F, A], dvalues [F], stats [8], loss_out (one element)); the
        gradients and loss_out are of S*L (S = *loss_scale for bfloat16 nets)."""
        cfg = cfg or LossCfg()
        b, keep, F, dev = self._batch(ro, env_ids, lengths, None, None, learner=True, inputs=False)
        _need(logits, torch.float32, "logits", F * self.A)
        _need(values, torch.float32, "values", F)
        c = L.LossCfg()
        c.clip, c.value_coef, c.entropy_coef = cfg.clip, cfg.value_coef, cfg.entropy_coef
        c.norm_adv = int(cfg.norm_adv)
        c.adv_stats = _ptr(adv_stats)
        if dlogits is None:
            dlogits = torch.empty(F, self.A, dtype=torch.float32, device=dev)
        if dvalues is None:
            dvalues = torch.empty(F, dtype=torch.float32, device=dev)
        if stats is None:
            stats = torch.empty(8, dtype=torch.float32, device=dev)
        if loss_out is None:
            loss_out = torch.empty((), dtype=torch.float32, device=dev)
        ws = self.workspace(L.PPO_OP_LOSS, F, len(env_ids), dev)
        check(lib().ppo_loss_head(self._h, C.byref(b), C.byref(c), _ptr(loss_scale), _ptr(logits), _ptr(values),
                                  _ptr(dlogits), _ptr(dvalues), _ptr(stats), _ptr(loss_out), _ptr(ws), ws.numel(),
                                  _stream(dev)), "ppo_loss_head")
        return dlogits, dvalues, stats, loss_out

    def loss_head_noalloc(self, ro, env_ids, lengths, logits, values, cfg: LossCfg = None, loss_scale=None,
                          adv_stats=None, dlogits=None, dvalues=None, stats=None, loss_out=None):
        """loss_head with the library's static scratch instead of a workspace
        (ppo_loss_head_noalloc); every output buffer must be given for a call
        that allocates nothing."""
        cfg = cfg or LossCfg()
        b, keep, F, dev = self._batch(ro, env_ids, lengths, None, None, learner=True, inputs=False)
        _need(logits, torch.float32, "logits", F * self.A)
        _need(values, torch.float32, "values", F)
        c = L.LossCfg()
        c.clip, c.value_coef, c.entropy_coef = cfg.clip, cfg.value_coef, cfg.entropy_coef
        c.norm_adv = int(cfg.norm_adv)
        c.adv_stats = _ptr(adv_stats)
        if dlogits is None:
            dlogits = torch.empty(F, self.A, dtype=torch.float32, device=dev)
        if dvalues is None:
            dvalues = torch.empty(F, dtype=torch.float32, device=dev)
        if stats is None:
            stats = torch.empty(8, dtype=torch.float32, device=dev)
        if loss_out is None:
            loss_out = torch.empty((), dtype=torch.float32, device=dev)
        check(lib().ppo_loss_head_noalloc(self._h, C.byref(b), C.byref(c), _ptr(loss_scale), _ptr(logits),
                                          _ptr(values), _ptr(dlogits), _ptr(dvalues), _ptr(stats), _ptr(loss_out),
                                          _stream(dev)), "ppo_loss_head_noalloc")
        return dlogits, dvalues, stats, loss_out

    def policy_backward(self, ro, env_ids, lengths, params, params_lp, dlogits, dvalues, grad=None):
        b, keep, F, dev = self._batch(ro, env_ids, lengths, params, params_lp, learner=False)
        _need(dlogits, torch.float32, "dlogits", F * self.A)
        _need(dvalues, torch.float32, "dvalues", F)
        if grad is None:
            grad = torch.empty(self.P, dtype=torch.float32, device=dev)
        ws = self.workspace(L.PPO_OP_LEARN, F, len(env_ids), dev)
        self._last_learn = (F, len(env_ids))
        check(lib().ppo_policy_backward(self._h, C.byref(b), _ptr(dlogits), _ptr(dvalues), _ptr(grad),
                                        _ptr(ws), ws.numel(), _stream(dev)), "ppo_policy_backward")
        return grad


    def policy_backward_ex(self, ro, env_ids, lengths, params, params_lp, dlogits, dvalues, grad=None,
                           dgoal=None):
        """ppo_policy_backward_ex: grad (parameter gradient, or None for a frozen
        net) and/or dgoal [F, 3] (goal-input gradient, 3-vector goal nets)."""
        b, keep, F, dev = self._batch(ro, env_ids, lengths, params, params_lp, learner=False)
        _need(dlogits, torch.float32, "dlogits", F * self.A)
        _need(dvalues, torch.float32, "dvalues", F)
        if grad is not None:
            _need(grad, torch.float32, "grad", self.P)
        if dgoal is not None:
            _need(dgoal, torch.float32, "dgoal", F * 3)
        ws = self.workspace(L.PPO_OP_LEARN, F, len(env_ids), dev)
        self._last_learn = (F, len(env_ids))
        check(lib().ppo_policy_backward_ex(self._h, C.byref(b), _ptr(dlogits), _ptr(dvalues), _ptr(grad),
                                           _ptr(dgoal), _ptr(ws), ws.numel(), _stream(dev)),
              "ppo_policy_backward_ex")
        return grad, dgoal

    def encode(self, obs, params, params_lp=None, out=None):
        """ppo_encode: features [F, flat] of frames obs [F, C, H, W]."""
        F = obs.shape[0]
        _need(obs, torch.bfloat16 if self.bf16 and self.spec.trunk != "none" else torch.float32, "obs")
        _need(params, torch.float32, "params", self.P)
        if self.bf16:
            _need(params_lp, torch.bfloat16, "params_lp", self.P)
        dev = obs.device
        out = torch.empty(F, self.flat, dtype=torch.float32, device=dev) if out is None else out
        _need(out, torch.float32, "out", F * self.flat)
        ws = self.workspace(L.PPO_OP_ACT, F, 1, dev)
        check(lib().ppo_encode(self._h, _ptr(obs), F, _ptr(params), _ptr(params_lp), _ptr(out), _ptr(ws),
                               ws.numel(), _stream(dev)), "ppo_encode")
        return out


def planner_goal(raw, dst=None, out=None, rows=None):
    """ppo_planner_goal: [ELU(r0) + 0.75, tanh(r1), tanh(r2)] of raw [F, ld]
    (first 3 columns) into row dst[f] (or f) of out [rows, 3]."""
    F, ld = raw.shape
    _need(raw, torch.float32, "raw")
    if dst is not None:
        _need(dst, torch.int32, "dst", F)
    if out is None:
        out = torch.zeros(rows or F, 3, dtype=torch.float32, device=raw.device)
    _need(out, torch.float32, "out")
    check(lib().ppo_planner_goal(_ptr(raw), ld, _ptr(dst), F, _ptr(out), _stream(raw.device)), "ppo_planner_goal")
    return out


def planner_goal_backward(raw, dgoal, out=None):
    """ppo_planner_goal_backward: d raw [F, ld] (first 3 columns) from dgoal [F, 3]."""
    F, ld = raw.shape
    _need(raw, torch.float32, "raw")
    _need(dgoal, torch.float32, "dgoal", F * 3)
    out = torch.zeros_like(raw) if out is None else out
    _need(out, torch.float32, "out", F * ld)
    check(lib().ppo_planner_goal_backward(_ptr(raw), ld, _ptr(dgoal), F, _ptr(out), _stream(raw.device)),
          "ppo_planner_goal_backward")
    return out


def gae(rew, val, done, lengths, gamma, lam, adv=None, ret=None, stats=None):
    """rew, done [T,N] (float32, uint8), val [T+1,N], lengths [N] int32 device or None."""
    T, N = rew.shape
    _need(rew, torch.float32, "rew")
    _need(val, torch.float32, "val", (T + 1) * N)
    _need(done, torch.uint8, "done", T * N)
    if lengths is not None:
        _need(lengths, torch.int32, "lengths", N)
    dev = rew.device
    adv = torch.empty(T, N, dtype=torch.float32, device=dev) if adv is None else adv
    ret = torch.empty(T, N, dtype=torch.float32, device=dev) if ret is None else ret
    check(lib().ppo_gae(_ptr(rew), _ptr(val), _ptr(done), _ptr(lengths), T, N, float(gamma), float(lam),
                        _ptr(adv), _ptr(ret), _ptr(stats), _stream(dev)), "ppo_gae")
    return adv, ret


class Adam:
    """Adam state (m, v, device scaler) for one flat parameter vector."""

    def __init__(self, P: int, device, lr=2.5e-4, betas=(0.9, 0.999), eps=1e-8, loss_scale=1.0,
                 growth_interval=0):
        self.P = P
        self.m = torch.zeros(P, dtype=torch.float32, device=device)
        self.v = torch.zeros(P, dtype=torch.float32, device=device)
        sc = L.Scaler()
        sc.scale = loss_scale
        raw = torch.frombuffer(bytearray(bytes(sc)), dtype=torch.uint8)
        self.scaler = raw.to(device)
        self.cfg = L.AdamCfg()
        self.cfg.lr, self.cfg.beta1, self.cfg.beta2, self.cfg.eps = lr, betas[0], betas[1], eps
        self.cfg.growth_interval = growth_interval
        self.ws = torch.empty(int(lib().ppo_adam_workspace_size(P)), dtype=torch.uint8, device=device)

    def loss_scale_ptr(self):
        return self.scaler  # float32 scale is the first field

    def scale_tensor(self):
        return self.scaler[:4].view(torch.float32)

    def state(self):
        raw = bytes(self.scaler.cpu().numpy().tobytes())
        sc = L.Scaler.from_buffer_copy(raw)
        return {"scale": sc.scale, "step": sc.step, "good_steps": sc.good_steps,
                "skipped": sc.skipped, "found_inf": sc.found_inf}

    def step(self, master, grad, lp_copy=None):
        _need(master, torch.float32, "master", self.P)
        _need(grad, torch.float32, "grad", self.P)
        if lp_copy is not None:
            _need(lp_copy, torch.bfloat16, "lp_copy", self.P)
        check(lib().ppo_adam_step(_ptr(master), _ptr(grad), _ptr(self.m), _ptr(self.v), _ptr(lp_copy),
                                  self.P, C.byref(self.cfg), _ptr(self.scaler), _ptr(self.ws),
                                  self.ws.numel(), _stream(master.device)), "ppo_adam_step")


def cast_bf16(src, dst=None):
    _need(src, torch.float32, "src")
    if dst is None:
        dst = torch.empty(src.shape, dtype=torch.bfloat16, device=src.device)
    check(lib().ppo_cast_bf16(_ptr(src), _ptr(dst), src.numel(), _stream(src.device)), "ppo_cast_bf16")
    return dst
