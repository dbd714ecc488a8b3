"""Workload descriptions for the DD-PPO worker hot path.

These are plain data: the network shape, the rollout shape and the PPO
hyper-parameters of each workload.  Nothing here computes any part of the
method.  Both the FP64 oracle and the HIP library are driven from these
descriptions, each with its own code.

Sources (DD-PPO, Wijmans et al., ICLR 2020):
  * 4 actions, 256x256 egocentric frames           -- Sec. 4 "Agent"
  * 2x2 AvgPool, ResNet50 with halved widths, GN     -- Sec. 4 "Agent", App. "Agent Design"
  * 1024x4x4 feature map -> 3x3 conv -> 128x4x4      -- App. "Agent Design", Visual Encoder
  * goal [d, theta] -> [d, cos, sin] -> FC-32        -- App. "Agent Design", Goal encoder
  * flatten 2048 -> FC hidden, prev-action emb 32,
    2-layer LSTM 512, softmax policy + value         -- App. "Agent Design", Navigation Policy
  * gamma 0.99, GAE tau 0.95, 128 steps x 4 envs,
    2 epochs x 2 minibatches, Adam 2.5e-4, no
    advantage normalisation                          -- Sec. 4 "Training"
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple


@dataclass(frozen=True)
class NetDesc:
    """Network shape.  trunk='tiny' is the two-conv encoder of the tiny
    workload; trunk='resnet' is the halved ResNet50 bottleneck layout;
    trunk='seresnext' the halved SE-ResNeXt50 one (bottleneck twice as wide,
    its 3x3 convolution split into `cardinality` groups, a squeeze-excite
    gate with reduction `se_reduction` on the residual branch)."""
    in_ch: int = 4
    in_hw: int = 256
    avgpool: bool = True
    trunk: str = "resnet"            # 'tiny' | 'resnet' | 'seresnext' | 'none' (in_ch-wide features in)
    tiny_ch: Tuple[int, int] = (16, 32)
    base_width: int = 32
    blocks: Tuple[int, int, int, int] = (3, 4, 6, 3)
    gn_groups: int = 16
    compress_ch: int = 128
    vis_hidden: int = 512
    goal_mode: str = "polar"         # 'raw' (2-vector concatenated) | 'polar' ([d,cos,sin] -> FC) |
                                     # 'vec3' (a given [magnitude, direction] 3-vector -> FC) | 'none
    goal_dim: int = 32               # width of the goal features fed to the LSTM
    prev_act_dim: int = 32           # 0: no previous-action embedding
    lstm_layers: int = 2
    hidden: int = 512
    num_actions: int = 4
    prev_actions: int = 0            # previous-action vocabulary (0: num_actions); + 1 start token
    cardinality: int = 16            # seresnext: groups of the 3x3 convolution
    se_reduction: int = 16           # seresnext: squeeze-excite hidden width = C / se_reduction

    # ---- derived shapes (pure bookkeeping) ----
    def mid_width(self, s: int) -> int:
        """Bottleneck width of stage s (output width 4 * base_width * 2**s)."""
        w = self.base_width << s
        return 2 * w if self.trunk == "seresnext" else w

    @property
    def enc_hw(self) -> int:
        """Spatial size after the optional 2x2 average pool."""
        return self.in_hw // 2 if self.avgpool else self.in_hw

    @property
    def feat_hw(self) -> int:
        """Spatial size of the map that is flattened into the visual FC."""
        if self.trunk == "none":
            return 1
        if self.trunk == "tiny":
            return self.enc_hw // 4
        return self.enc_hw // 32

    @property
    def feat_ch(self) -> int:
        if self.trunk == "none":
            return self.in_ch
        return self.tiny_ch[1] if self.trunk == "tiny" else self.compress_ch

    @property
    def flat_dim(self) -> int:
        return self.feat_ch * self.feat_hw * self.feat_hw

    @property
    def emb_rows(self) -> int:
        """Rows of the previous-action embedding: every action and the start token."""
        return (self.prev_actions or self.num_actions) + 1

    @property
    def lstm_in(self) -> int:
        return self.vis_hidden + self.goal_dim + self.prev_act_dim


def controller_nets(agent: NetDesc, plan_hidden: int = 512):
    """The two features-in nets of the neural-controller system built on a
    trained agent (Sec. 6, appendix "Neural controller additional details"):
    the controller core (the agent's policy core, its goal FC fed a given
    [magnitude, direction] 3-vector) and the planner (the same policy layout
    with a plan_hidden-wide visual FC and LSTM, no goal input, the agent's
    previous actions, and 3 head outputs besides the value)."""
    if agent.goal_mode != "polar":
        raise ValueError("the controller's goal FC must read a 3-vector (polar goal agents)")
    feat = dict(trunk="none", in_ch=agent.flat_dim, in_hw=1, avgpool=False)
    ctrl = replace(agent, goal_mode="vec3", **feat)
    plan = replace(agent, goal_mode="none", goal_dim=0, num_actions=3, prev_actions=agent.num_actions,
                   hidden=plan_hidden, vis_hidden=plan_hidden, **feat)
    return ctrl, plan


@dataclass(frozen=True)
class PPOCfg:
    gamma: float = 0.99
    lam: float = 0.95
    clip: float = 0.2
    value_coef: float = 0.5
    entropy_coef: float = 0.01
    lr: float = 2.5e-4
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    epochs: int = 2
    minibatches: int = 2
    norm_adv: bool = False


@dataclass(frozen=True)
class Workload:
    name: str
    net: NetDesc
    T: int
    N: int
    dtype: str = "f32"               # 'f32' | 'bf16'
    ragged: bool = False             # lengths ~ U{T/4 .. T}
    ppo: PPOCfg = field(default_factory=PPOCfg)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


TINY_NET = NetDesc(in_hw=32, avgpool=False, trunk="tiny", gn_groups=8,
                   vis_hidden=64, goal_mode="raw", goal_dim=2, prev_act_dim=0,
                   lstm_layers=1, hidden=64)
RESNET_NET = NetDesc()
RESNET_NET_128 = NetDesc(in_hw=128)
SERESNEXT_NET = NetDesc(trunk="seresnext")
# the paper's largest agent: SE-ResNeXt101 (halved) and a 2 x 1024 LSTM, the
# visual FC mapping to the hidden size
SERESNEXT101_NET = NetDesc(trunk="seresnext", blocks=(3, 4, 23, 3), vis_hidden=1024, hidden=1024)

# The five workloads: tiny FP32; paper-shaped worker in FP32 and in BF16;
# the differentiation form at 128x128 frames; the ragged batching form.
C0 = Workload("tiny_f32_T16_N2", TINY_NET, T=16, N=2, dtype="f32",
              ppo=PPOCfg(epochs=1, minibatches=1))
C1 = Workload("resnet50h_f32_T128_N4", RESNET_NET, T=128, N=4, dtype="f32")
C2 = Workload("resnet50h_bf16_T128_N4", RESNET_NET, T=128, N=4, dtype="bf16")
C3 = Workload("resnet50h_bf16_128px_T128_N16", RESNET_NET_128, T=128, N=16, dtype="bf16")
C4 = Workload("resnet50h_bf16_ragged_T128_N64", RESNET_NET, T=128, N=64, dtype="bf16",
              ragged=True)
# the SE-ResNeXt50 encoder (halved widths) in the default worker configuration
C5 = Workload("seresnext50h_bf16_T128_N4", SERESNEXT_NET, T=128, N=4, dtype="bf16")
C6 = Workload("seresnext101h_lstm1024_bf16_T128_N4", SERESNEXT101_NET, T=128, N=4, dtype="bf16")

WORKLOADS = {"C0": C0, "C1": C1, "C2": C2, "C3": C3, "C4": C4, "C5": C5, "C6": C6}
