"""ppo_loss_head_noalloc (the loss head on the library's static scratch)
against ppo_loss_head (caller's workspace) on the same inputs: identical
outputs on two calls in a row, the second with fewer frames, for a float32
net and a bfloat16 net with a loss scale and advantage normalisation; a
minibatch beyond the static maximum is refused on the host."""
import numpy as np
import pytest
import torch

from paper_1911_00357_amd._lib import PPO_ESHAPE, PPOError
from tests.gpu_util import DEV, random_record, to_device
from tests.nets import TINY_PLUS

pytestmark = pytest.mark.gpu


def _case(P, dtype, T, N, lengths, envs, seed, norm_adv):
    n = P.Net(TINY_PLUS, dtype)
    rec = random_record(TINY_PLUS, T, N, seed, lengths=lengths)
    ro = to_device(rec)
    F = int(sum(rec["lengths"][e] for e in envs))
    g = torch.Generator(device="cpu").manual_seed(seed)
    logits = torch.randn(F, n.A, generator=g).to(DEV)
    values = torch.randn(F, generator=g).to(DEV)
    cfg = P.LossCfg(norm_adv=norm_adv)
    adv_stats = None
    if norm_adv:
        a = rec["adv"]
        adv_stats = torch.tensor([a.mean(), a.var()], dtype=torch.float64, device=DEV)
    scale = torch.tensor([1024.0], device=DEV) if dtype == "bf16" else None
    lens = rec["lengths"] if lengths is not None else None
    ref = n.loss_head(ro, envs, lens, logits, values, cfg, scale, adv_stats)
    got = n.loss_head_noalloc(ro, envs, lens, logits, values, cfg, scale, adv_stats)
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("dtype,norm_adv", [("f32", False), ("bf16", True)])
def test_noalloc_loss_head_matches_loss_head(P, dtype, norm_adv):
    print(f"no-alloc loss head {dtype} norm_adv={norm_adv}", flush=True)
    calls = [(12, 6, [12, 9, 7, 12, 3, 5], [0, 1, 2, 3, 4, 5], 1),   # 48 frames
             (5, 3, [5, 2, 4], [2, 0], 2)]                          # then 9 frames
    for T, N, lengths, envs, seed in calls:
        ref, got = _case(P, dtype, T, N, lengths, envs, seed, norm_adv)
        for name, a, b in zip(("dlogits", "dvalues", "stats", "loss"), ref, got):
            assert torch.equal(a, b), name
        assert torch.isfinite(got[2]).all() and got[0].abs().sum() > 0


def test_noalloc_loss_head_refuses_beyond_its_scratch(P):
    from paper_1911_00357_amd._lib import lib as _lib
    cap = int(_lib().ppo_loss_head_noalloc_max_frames())
    n = P.Net(TINY_PLUS, "f32")
    T, N = cap // 2 + 1, 2                                           # 2 envs of T steps > cap frames
    ro = {"mask": torch.ones(T + 1, N, device=DEV),
          "action": torch.zeros(T + 1, N, dtype=torch.int32, device=DEV),
          "logp": torch.zeros(T + 1, N, device=DEV), "adv": torch.zeros(T, N, device=DEV),
          "ret": torch.zeros(T, N, device=DEV)}
    F = T * N
    logits = torch.zeros(F, n.A, device=DEV)
    values = torch.zeros(F, device=DEV)
    with pytest.raises(PPOError) as e:
        n.loss_head_noalloc(ro, [0, 1], None, logits, values)
    assert e.value.status == PPO_ESHAPE
