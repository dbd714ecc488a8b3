"""The SE-ResNeXt50 encoder (halved widths; Sec. 6, Table 1; App. "Agent
Design") on the GPU against the float64 oracle: act steps and learner
minibatches with the same bars as the ResNet (tests/test_gpu_parity.py),
the GPU's ReLU / max-pool / squeeze-excite decisions imposed and validated;
and the grouped-convolution kernels alone against the oracle's grouped
convolution, forward and both gradients, at every stage's width."""
import numpy as np
import pytest
import torch

from oracle import nn as onn
from synth import rollout as R
from synth.configs import C5, C6
from tests.gpu_util import assert_close
from tests.nets import MINI_SERESNEXT, SERESNEXT_64
from tests.test_gpu_parity import GN_FORMS, _act_case, _loss_case, check_act, check_loss, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,net,dtype,B", [("mini_seresnext", MINI_SERESNEXT, "f32", 4),
                                              ("mini_seresnext", MINI_SERESNEXT, "bf16", 4),
                                              ("seresnext64", SERESNEXT_64, "f32", 2),
                                              ("seresnext64", SERESNEXT_64, "bf16", 3)])
def test_act_parity_seresnext(P, name, net, dtype, B):
    say(f"act {name} {dtype} B={B}")
    out, ref = _act_case(P, net, dtype, B, seed=B + 20)
    check_act(out, ref, dtype, B, name)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_act_parity_seresnext_paper_shape(P, dtype):
    """SE-ResNeXt50 (halved) at 256x256 frames, batch 4."""
    say(f"act seresnext paper shape {dtype}")
    out, ref = _act_case(P, C5.net, dtype, 4, seed=31, state_rows=5)
    check_act(out, ref, dtype, 4, "seresnext")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_act_parity_seresnext101_lstm1024(P, dtype):
    """The paper's largest agent (SE-ResNeXt101 halved, 2 x 1024 LSTM) at
    256x256 frames, batch 4; its core takes the per-layer step kernel."""
    say(f"act seresnext101 + 1024-d LSTM {dtype}")
    out, ref = _act_case(P, C6.net, dtype, 4, seed=33)
    check_act(out, ref, dtype, 4, "seresnext101")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_loss_backward_parity_mini_seresnext(P, dtype):
    say(f"loss {dtype} mini_seresnext")
    c = _loss_case(P, MINI_SERESNEXT, dtype, 5, 3, [2, 1, 0], [5, 3, 4], seed=41, same_decisions=True)
    check_loss(MINI_SERESNEXT, dtype, c, "mini_seresnext")


@pytest.mark.parametrize("form", ["default", "partial"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_loss_backward_seresnext_paper_shape(P, dtype, form, monkeypatch):
    """SE-ResNeXt50 (halved) at 256x256 frames: 2 envs x (4, 2) steps."""
    for k, v in GN_FORMS[form].items():
        monkeypatch.setenv(k, v)
    say(f"loss seresnext paper shape {dtype}, GroupNorm {form}")
    c = _loss_case(P, C5.net, dtype, 4, 3, [2, 0], [4, 2, 3], seed=43, same_decisions=True)
    check_loss(C5.net, dtype, c, f"seresnext {form}")


# ------------------------------------------------- the grouped convolution
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_grouped_conv_units_match_oracle(P, dtype, monkeypatch):
    """Every grouped 3x3 of the paper-width SE-ResNeXt (16 groups of 4, 8, 16
    and 32 channels; stride 2 on the first block of stages 1-3) on 3 frames:
    forward, data gradient and weight gradient through the benchmark entry
    (the kernels the encoder runs), against the oracle's grouped convolution
    on the same operands; bfloat16 operands rounded as the kernels round
    them (each product exact in float32)."""
    from paper_1911_00357_amd import api
    from paper_1911_00357_amd._lib import PPO_OP_LEARN
    monkeypatch.setattr(api, "POISON_WS", False)   # the operands are written into the workspace first
    net = C5.net
    n = P.Net(net, dtype)
    F = 3
    flat = R.init_params(net, 5)
    params = torch.tensor(flat, device="cuda")
    lp = P.cast_bf16(params) if dtype == "bf16" else None
    grad = torch.zeros_like(params)
    ws = n.workspace(PPO_OP_LEARN, F, 1, params.device)   # the buffer bench_unit_gemm uses
    off = {name: (o, cnt) for name, o, cnt in n.tensors()}
    g = np.random.default_rng(7)
    tol = 1e-5
    done = set()
    nunits = n.probe(PPO_OP_LEARN, F, 1, 3)[3][0]
    rnd = onn.round_bf16 if dtype == "bf16" else (lambda a: a)
    for u in range(nunits):
        name, _, _, (ho, wo, co, _) = n.probe(PPO_OP_LEARN, F, 1, 0, u)
        if not name.endswith(".c2"):
            continue
        s_, j = int(name.split(".")[1][1:]), int(name.split(".")[2][1:])
        stride = 2 if (j == 0 and s_ > 0) else 1
        key = (co, stride)
        if key in done:
            continue
        done.add(key)
        Gr = net.cardinality
        cg = co // Gr
        hi = ho * stride
        say(f"grouped conv {name}: {co} channels in {Gr} groups, {hi}x{hi} -> {ho}x{wo}, {dtype}")
        # operands: X (unit input, NHWC) at scratch 'ga', DY (output gradient) at 'gb'
        x = g.standard_normal((F, hi, hi, co)).astype(np.float32)
        dy = g.standard_normal((F, ho, wo, co)).astype(np.float32)
        offs = _scratch_offsets(n, F)
        _put(ws, offs["ga"], x)
        _put(ws, offs["gb"], dy)
        o, cnt = off[name]
        w = flat[o:o + cnt].reshape(co, 3, 3, cg)
        if dtype == "bf16":
            w = R.round_bf16(w)
        w_oihw = w.transpose(0, 3, 1, 2).astype(np.float64)
        x_nchw = x.transpose(0, 3, 1, 2).astype(np.float64)
        dy_nchw = dy.transpose(0, 3, 1, 2).astype(np.float64)
        y_ref = onn.conv2d_grouped(rnd(x_nchw), w_oihw, stride, 1, Gr)
        dx_ref, dw_ref = onn.conv2d_grouped_backward(rnd(x_nchw), w_oihw, stride, 1, dy_nchw, Gr)
        # forward -> 'gu'
        n.bench_unit_gemm(0, u, F, params, lp, grad, 1)
        torch.cuda.synchronize()
        y = _get(ws, offs["gu"], F * ho * wo * co).reshape(F, ho, wo, co).transpose(0, 3, 1, 2)
        assert_close(name + " forward", y, y_ref, tol)
        # data gradient -> 'gu'
        n.bench_unit_gemm(1, u, F, params, lp, grad, 1)
        torch.cuda.synchronize()
        dx = _get(ws, offs["gu"], F * hi * hi * co).reshape(F, hi, hi, co).transpose(0, 3, 1, 2)
        assert_close(name + " data gradient", dx, dx_ref, tol)
        # weight gradient -> grad slot (O, KH, KW, I/G as stored)
        n.bench_unit_gemm(2, u, F, params, lp, grad, 1)
        torch.cuda.synchronize()
        dw = grad[o:o + cnt].cpu().numpy().reshape(co, 3, 3, cg).transpose(0, 3, 1, 2)
        assert_close(name + " weight gradient", dw, dw_ref, tol)
    assert len(done) == 7        # 4 stages, strides 1 and 2 (stage 0 has no stride-2 block)


def _scratch_offsets(n, F):
    """Byte offsets of ppo_bench_unit_gemm's operand buffers in a learner
    workspace: input X ('ga'), output gradient DY ('gb'), output ('gu')."""
    from paper_1911_00357_amd._lib import PPO_OP_LEARN
    return {k: n.probe(PPO_OP_LEARN, F, 1, 9, i)[2] for i, k in enumerate(("ga", "gb", "gu"))}


def _put(ws, off, a):
    b = torch.from_numpy(np.ascontiguousarray(a, np.float32).view(np.uint8).reshape(-1))
    ws[off:off + b.numel()].copy_(b.to(ws.device))


def _get(ws, off, n):
    return ws[off:off + 4 * n].view(torch.float32).cpu().numpy().astype(np.float64)
