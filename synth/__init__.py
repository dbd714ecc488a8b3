"""Seeded synthetic workloads (shapes, hyper-parameters, input streams).

Shared by the oracle, the tests and the benchmark; holds none of the
method's arithmetic."""
from .configs import NetDesc, PPOCfg, Workload, WORKLOADS, C0, C1, C2, C3, C4, C5, C6, TINY_NET, RESNET_NET, SERESNEXT_NET
from .layout import tensor_list, param_count
from . import rollout
