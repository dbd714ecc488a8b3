"""MI355X (gfx950) hot path of one DD-PPO worker: batched act step, GAE,
PPO loss + hand-written backward, Adam -- a C ABI over HIP kernels
(include/ddppo.h) with a thin torch binding."""
from ._lib import lib, PPOError  # noqa: F401
from .api import Net, LossCfg, Adam, gae, cast_bf16, planner_goal, planner_goal_backward  # noqa: F401
