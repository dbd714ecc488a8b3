"""ctypes declarations of the C ABI in include/ddppo.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddppo.so")

c_int, c_float, c_size_t, c_void_p = C.c_int, C.c_float, C.c_size_t, C.c_void_p
P_i32 = C.POINTER(C.c_int32)

PPO_OK, PPO_EINVAL, PPO_ESHAPE, PPO_EUNSUPPORTED, PPO_EWORKSPACE, PPO_EDEVICE = 0, -1, -2, -3, -4, -5
PPO_F32, PPO_BF16 = 0, 1
PPO_TRUNK_TINY, PPO_TRUNK_RESNET, PPO_TRUNK_SERESNEXT, PPO_TRUNK_NONE = 0, 1, 2, 3
PPO_GOAL_RAW, PPO_GOAL_POLAR, PPO_GOAL_VEC3, PPO_GOAL_NONE = 0, 1, 2, 3
PPO_OP_ACT, PPO_OP_LEARN, PPO_OP_LOSS = 0, 1, 2
PPO_TIMER_ALL_UNITS = -2
PPO_COLLECT_GRAPH, PPO_COLLECT_TRIM = 1, 2

STATUS_NAMES = {0: "PPO_OK", -1: "PPO_EINVAL", -2: "PPO_ESHAPE", -3: "PPO_EUNSUPPORTED",
                -4: "PPO_EWORKSPACE", -5: "PPO_EDEVICE"}


class NetDesc(C.Structure):
    _fields_ = [("in_ch", c_int), ("in_hw", c_int), ("avgpool", c_int), ("trunk", c_int),
                ("tiny_ch", c_int * 2), ("base_width", c_int), ("blocks", c_int * 4),
                ("gn_groups", c_int), ("compress_ch", c_int), ("vis_hidden", c_int),
                ("goal_mode", c_int), ("goal_dim", c_int), ("prev_act_dim", c_int),
                ("lstm_layers", c_int), ("hidden", c_int), ("num_actions", c_int), ("dtype", c_int),
                ("cardinality", c_int), ("se_reduction", c_int), ("prev_actions", c_int)]


class ActIO(C.Structure):
    _fields_ = [("batch", c_int), ("state_rows", c_int), ("obs", c_void_p), ("goal", c_void_p), ("prev_action", c_void_p),
                ("mask", c_void_p), ("h_in", c_void_p), ("c_in", c_void_p), ("u", c_void_p),
                ("params", c_void_p), ("params_lp", c_void_p), ("action", c_void_p),
                ("logp", c_void_p), ("value", c_void_p), ("h_out", c_void_p), ("c_out", c_void_p),
                ("logits", c_void_p), ("active", c_void_p)]


class CollectIO(C.Structure):
    _fields_ = [("T", c_int), ("N", c_int), ("t_begin", c_int), ("t_end", c_int), ("obs", c_void_p),
                ("goal", c_void_p), ("mask", c_void_p), ("u", c_void_p), ("active", c_void_p), ("lengths", P_i32),
                ("params", c_void_p), ("params_lp", c_void_p), ("actions", c_void_p), ("logp", c_void_p),
                ("value", c_void_p), ("h_hist", c_void_p), ("c_hist", c_void_p), ("h_last", c_void_p),
                ("c_last", c_void_p)]


class Batch(C.Structure):
    _fields_ = [("T", c_int), ("N", c_int), ("nb", c_int), ("env_ids", P_i32), ("lengths", P_i32),
                ("obs", c_void_p), ("goal", c_void_p), ("prev_action", c_void_p), ("mask", c_void_p),
                ("action", c_void_p), ("logp_old", c_void_p), ("adv", c_void_p), ("ret", c_void_p),
                ("h0", c_void_p), ("c0", c_void_p), ("params", c_void_p), ("params_lp", c_void_p)]


class LossCfg(C.Structure):
    _fields_ = [("clip", c_float), ("value_coef", c_float), ("entropy_coef", c_float),
                ("norm_adv", c_int), ("adv_stats", c_void_p)]


class AdamCfg(C.Structure):
    _fields_ = [("lr", c_float), ("beta1", c_float), ("beta2", c_float), ("eps", c_float),
                ("growth_interval", c_int)]


class Scaler(C.Structure):
    _fields_ = [("scale", c_float), ("step", C.c_int32), ("good_steps", C.c_int32),
                ("skipped", C.c_int32), ("found_inf", C.c_int32), ("pad", C.c_int32 * 3)]


EXPORTS = {
    "ppo_net_create": (c_int, [C.POINTER(NetDesc), C.POINTER(c_void_p)]),
    "ppo_net_destroy": (None, [c_void_p]),
    "ppo_param_count": (c_size_t, [c_void_p]),
    "ppo_param_tensor": (c_int, [c_void_p, c_int, C.POINTER(C.c_char_p), C.POINTER(c_size_t),
                                 C.POINTER(c_size_t)]),
    "ppo_workspace_size": (c_int, [c_void_p, c_int, c_int, c_int, C.POINTER(c_size_t)]),
    "ppo_act": (c_int, [c_void_p, C.POINTER(ActIO), c_void_p, c_size_t, c_void_p]),
    "ppo_collect": (c_int, [c_void_p, C.POINTER(CollectIO), c_int, c_void_p, c_size_t, c_void_p]),
    "ppo_collect_clear": (c_int, [c_void_p]),
    "ppo_collect_graph_count": (c_int, [c_void_p]),
    "ppo_gae": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_float, c_float,
                        c_void_p, c_void_p, c_void_p, c_void_p]),
    "ppo_loss_backward": (c_int, [c_void_p, C.POINTER(Batch), C.POINTER(LossCfg), c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_size_t, c_void_p]),
    "ppo_policy_forward": (c_int, [c_void_p, C.POINTER(Batch), c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_size_t, c_void_p]),
    "ppo_policy_backward": (c_int, [c_void_p, C.POINTER(Batch), c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_size_t, c_void_p]),
    "ppo_policy_backward_ex": (c_int, [c_void_p, C.POINTER(Batch), c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_void_p, c_size_t, c_void_p]),
    "ppo_encode": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ppo_planner_goal": (c_int, [c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p]),
    "ppo_planner_goal_backward": (c_int, [c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p]),
    "ppo_loss_head": (c_int, [c_void_p, C.POINTER(Batch), C.POINTER(LossCfg), c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ppo_loss_head_noalloc": (c_int, [c_void_p, C.POINTER(Batch), C.POINTER(LossCfg), c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ppo_loss_head_noalloc_max_frames": (c_size_t, []),
    "ppo_adam_workspace_size": (c_size_t, [c_size_t]),
    "ppo_adam_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                              C.POINTER(AdamCfg), c_void_p, c_void_p, c_size_t, c_void_p]),
    "ppo_cast_bf16": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "ppo_workspace_probe": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, C.POINTER(C.c_char_p),
                                    C.POINTER(c_int), C.POINTER(c_size_t), C.POINTER(c_int)]),
    "ppo_bench_unit_gemm": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_size_t, c_int, C.POINTER(C.c_double), c_void_p]),
    "ppo_autotune": (c_int, [c_void_p, c_int, C.POINTER(c_int)]),
    "ppo_autotune_table": (c_int, [c_void_p, c_int, C.POINTER(C.c_int64), c_int, C.POINTER(c_int)]),
    "ppo_gemm_timer_arm": (c_int, [c_void_p, c_int, c_int, c_int]),
    "ppo_gemm_timer_read": (c_int, [c_void_p, C.POINTER(c_int), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]),
    "ppo_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """Load libddppo.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1911_00357_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class PPOError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().ppo_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, where: str):
    if status != PPO_OK:
        raise PPOError(status, where)
