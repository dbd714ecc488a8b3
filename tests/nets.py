"""Small network variants used by the gradient and parity tests; together
they reach every branch of the agent (tiny trunk, bottleneck trunk with
projection and identity shortcuts, max pool, goal FC, previous-action
embedding, stacked LSTM)."""
from synth.configs import NetDesc, PPOCfg, Workload, TINY_NET

TINY_PLUS = NetDesc(in_hw=32, avgpool=False, trunk="tiny", gn_groups=8, vis_hidden=16,
                    goal_mode="polar", goal_dim=8, prev_act_dim=8, lstm_layers=2, hidden=16)

MINI_RESNET = NetDesc(in_hw=64, avgpool=True, trunk="resnet", base_width=4, blocks=(1, 2, 1, 1),
                      gn_groups=2, compress_ch=8, vis_hidden=16, goal_mode="polar", goal_dim=8,
                      prev_act_dim=8, lstm_layers=2, hidden=16)

# the SE-ResNeXt trunk at small widths: 2 groups in every 3x3, SE hidden width C/4
MINI_SERESNEXT = NetDesc(in_hw=64, avgpool=True, trunk="seresnext", base_width=4, blocks=(1, 2, 1, 1),
                         gn_groups=2, compress_ch=8, vis_hidden=16, goal_mode="polar", goal_dim=8,
                         prev_act_dim=8, lstm_layers=2, hidden=16, cardinality=2, se_reduction=4)
# the real SE-ResNeXt widths (16 groups, reduction 16) on a 64x64 frame
SERESNEXT_64 = NetDesc(in_hw=64, trunk="seresnext")
# a bottleneck trunk with the real widths but a 64x64 frame (feature map 1x1)
RESNET_64 = NetDesc(in_hw=64)
# the real trunk with a small core, and the tiny trunk with the real core
RESNET_SMALLCORE = NetDesc(in_hw=64, vis_hidden=16, goal_dim=8, prev_act_dim=8, hidden=16)
TINY_BIGCORE = NetDesc(in_hw=32, avgpool=False, trunk="tiny", gn_groups=8, vis_hidden=512,
                       goal_mode="polar", goal_dim=32, prev_act_dim=32, lstm_layers=2, hidden=512)
# the 1024-unit LSTM variant of the paper's larger agents (tiny trunk)
TINY_CORE1024 = NetDesc(in_hw=32, avgpool=False, trunk="tiny", gn_groups=8, vis_hidden=512,
                        goal_mode="polar", goal_dim=32, prev_act_dim=32, lstm_layers=2, hidden=1024)


def wl(net, T=4, N=3, dtype="f32", ragged=False, **ppo):
    return Workload("test", net, T=T, N=N, dtype=dtype, ragged=ragged,
                    ppo=PPOCfg(**ppo) if ppo else PPOCfg())


__all__ = ["TINY_NET", "TINY_PLUS", "MINI_RESNET", "MINI_SERESNEXT", "RESNET_64", "SERESNEXT_64", "wl"]
