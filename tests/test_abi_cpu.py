"""The C-ABI library loads, exports every symbol the header declares, agrees
with the flat parameter format, and rejects bad arguments with a status
before touching the GPU (runs without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from paper_1911_00357_amd import _lib as L
from synth.layout import tensor_list
from tests.nets import MINI_RESNET, MINI_SERESNEXT, SERESNEXT_64, TINY_BIGCORE, TINY_PLUS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddppo.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ppo_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS), set(names) ^ set(L.EXPORTS)


def test_struct_layouts_match_header(tmp_path):
    """Compile the header with the host C compiler and compare every struct's
    size and field offsets with the binding's ctypes declarations."""
    import subprocess
    pairs = {"ppo_net_desc": L.NetDesc, "ppo_act_io": L.ActIO, "ppo_collect_io": L.CollectIO, "ppo_batch": L.Batch,
             "ppo_loss_cfg": L.LossCfg, "ppo_adam_cfg": L.AdamCfg, "ppo_scaler": L.Scaler}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void){']
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in pairs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("wl", ["C0", "C1", "C3", "C5"])
def test_param_layout_matches_generator(wl):
    import paper_1911_00357_amd as P
    net = synth.WORKLOADS[wl].net
    n = P.Net(net, synth.WORKLOADS[wl].dtype)
    got = [(off, cnt) for name, off, cnt in n.tensors()]
    exp = [(t.offset, int(np.prod(t.shape))) for t in tensor_list(net)]
    assert got == exp
    assert n.P == synth.param_count(net)


@pytest.mark.parametrize("net", [TINY_PLUS, MINI_RESNET, TINY_BIGCORE, MINI_SERESNEXT, SERESNEXT_64])
def test_test_nets_create(net):
    import paper_1911_00357_amd as P
    assert P.Net(net, "f32").P == synth.param_count(net)
    n = P.Net(net, "bf16")
    assert n.P == synth.param_count(net)
    got = [(off, cnt) for name, off, cnt in n.tensors()]
    assert got == [(t.offset, int(np.prod(t.shape))) for t in tensor_list(net)]


@pytest.mark.parametrize("bad", [dict(cardinality=0), dict(cardinality=3), dict(se_reduction=0),
                                 dict(se_reduction=7), dict(cardinality=1)])
def test_seresnext_create_rejects_bad_groups(bad):
    """Groups that do not divide the bottleneck, a reduction that does not
    divide the block width, or a grouped 3x3 too wide for the direct kernels
    (one group: 512 channels per group) are refused before anything runs."""
    import paper_1911_00357_amd.api as A
    lib = L.lib()
    d = A.desc_from(synth.C5.net, "bf16")
    for k, v in bad.items():
        setattr(d, k, v)
    h = C.c_void_p()
    assert lib.ppo_net_create(C.byref(d), C.byref(h)) == L.PPO_ESHAPE
    assert not h.value


def _desc(**kw):
    import paper_1911_00357_amd.api as A
    d = A.desc_from(synth.C1.net, "f32")
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("bad", [dict(gn_groups=7), dict(in_hw=100), dict(num_actions=9),
                                 dict(trunk=5), dict(dtype=3), dict(lstm_layers=0),
                                 dict(goal_mode=0)])
def test_net_create_rejects_bad_descriptions(bad):
    lib = L.lib()
    h = C.c_void_p()
    st = lib.ppo_net_create(C.byref(_desc(**bad)), C.byref(h))
    assert st in (L.PPO_ESHAPE, L.PPO_EINVAL)
    assert not h.value
    assert len(lib.ppo_last_error()) > 0


def test_calls_reject_null_and_bad_sizes_before_any_launch():
    lib = L.lib()
    h = C.c_void_p()
    assert lib.ppo_net_create(C.byref(_desc()), C.byref(h)) == L.PPO_OK
    try:
        assert lib.ppo_net_create(None, C.byref(h)) == L.PPO_EINVAL
        io = L.ActIO()
        io.batch = 4
        assert lib.ppo_act(h, C.byref(io), None, 0, None) == L.PPO_EINVAL   # null pointers
        io.batch = 0
        assert lib.ppo_act(h, C.byref(io), None, 0, None) == L.PPO_ESHAPE
        b = C.c_size_t()
        assert lib.ppo_workspace_size(h, L.PPO_OP_LEARN, 0, 1, C.byref(b)) == L.PPO_ESHAPE
        assert lib.ppo_workspace_size(h, L.PPO_OP_LEARN, 64, 300, C.byref(b)) == L.PPO_ESHAPE
        assert lib.ppo_workspace_size(h, 7, 64, 1, C.byref(b)) == L.PPO_EINVAL
        assert lib.ppo_workspace_size(h, L.PPO_OP_ACT, 4, 1, C.byref(b)) == L.PPO_OK and b.value > 0
        # act with every pointer set but a workspace that is too small
        fake = C.c_void_p(256)
        io = L.ActIO()
        io.batch = 4
        for f in ("obs", "goal", "prev_action", "mask", "h_in", "c_in", "u", "params", "action", "logp",
                  "value", "h_out", "c_out"):
            setattr(io, f, fake)
        assert lib.ppo_act(h, C.byref(io), fake, 16, None) == L.PPO_EWORKSPACE
        io.state_rows = 2
        assert lib.ppo_act(h, C.byref(io), fake, 1 << 40, None) == L.PPO_ESHAPE
        assert lib.ppo_gae(None, None, None, None, 4, 4, 0.99, 0.95, None, None, None, None) == L.PPO_EINVAL
        assert lib.ppo_gae(fake, fake, fake, None, 0, 4, 0.99, 0.95, fake, fake, None, None) == L.PPO_ESHAPE
        assert lib.ppo_gae(fake, fake, fake, None, 4, 4, 1.5, 0.95, fake, fake, None, None) == L.PPO_EINVAL
        # loss backward: env id out of range, length out of range
        bt = L.Batch()
        bt.T, bt.N, bt.nb = 8, 4, 2
        ids = (C.c_int32 * 2)(0, 9)
        bt.env_ids = C.cast(ids, L.P_i32)
        for f in ("obs", "goal", "prev_action", "mask", "action", "logp_old", "adv", "ret", "h0", "c0",
                  "params"):
            setattr(bt, f, fake)
        cfg = L.LossCfg()
        assert lib.ppo_loss_backward(h, C.byref(bt), C.byref(cfg), None, fake, fake, fake, 1 << 40,
                                     None) == L.PPO_ESHAPE
        ids[1] = 1
        lens = (C.c_int32 * 4)(8, 9, 8, 8)
        bt.lengths = C.cast(lens, L.P_i32)
        assert lib.ppo_loss_backward(h, C.byref(bt), C.byref(cfg), None, fake, fake, fake, 1 << 40,
                                     None) == L.PPO_ESHAPE
        lens[1] = 8
        assert lib.ppo_loss_backward(h, C.byref(bt), C.byref(cfg), None, fake, fake, fake, 64,
                                     None) == L.PPO_EWORKSPACE
        # Adam: bad hyper-parameters and small workspace
        ac = L.AdamCfg()
        ac.lr, ac.beta1, ac.beta2, ac.eps = 1e-3, 0.9, 0.999, 1e-8
        assert lib.ppo_adam_step(fake, fake, fake, fake, None, 10, C.byref(ac), fake, fake, 4, None) \
            == L.PPO_EWORKSPACE
        ac.beta1 = 1.5
        assert lib.ppo_adam_step(fake, fake, fake, fake, None, 10, C.byref(ac), fake, fake, 1 << 20, None) \
            == L.PPO_EINVAL
        # probe
        name, relu, off = C.c_char_p(), C.c_int(), C.c_size_t()
        dims = (C.c_int * 4)()
        assert lib.ppo_workspace_probe(h, 1, 8, 2, 0, 999, C.byref(name), C.byref(relu), C.byref(off), dims) \
            == L.PPO_EINVAL
        assert lib.ppo_workspace_probe(h, 1, 8, 2, 3, 0, None, None, C.byref(off), dims) == L.PPO_OK
        assert dims[0] == 54
    finally:
        lib.ppo_net_destroy(h)


def test_collect_rejects_bad_arguments_before_any_launch():
    """ppo_collect's host checks: step range, null buffers, unknown flags,
    unordered or out-of-range lengths, and the per-step ppo_act checks
    (workspace size) of its largest step; an empty step range is a no-op.
    Nothing here reaches a HIP call."""
    lib = L.lib()
    h = C.c_void_p()
    assert lib.ppo_net_create(C.byref(_desc()), C.byref(h)) == L.PPO_OK
    try:
        fake = C.c_void_p(256)
        io = L.CollectIO()
        io.T, io.N, io.t_begin, io.t_end = 8, 4, 0, 9
        assert lib.ppo_collect(h, C.byref(io), 0, fake, 1 << 40, None) == L.PPO_EINVAL   # null buffers
        for f in ("obs", "goal", "mask", "u", "params", "actions", "logp", "value", "h_hist", "c_hist",
                  "h_last", "c_last"):
            setattr(io, f, fake)
        assert lib.ppo_collect(h, C.byref(io), 0, fake, 16, None) == L.PPO_EWORKSPACE
        assert lib.ppo_collect(h, C.byref(io), 8, fake, 1 << 40, None) == L.PPO_EINVAL   # unknown flag
        io.t_end = 10
        assert lib.ppo_collect(h, C.byref(io), 0, fake, 1 << 40, None) == L.PPO_ESHAPE
        io.t_begin, io.t_end = 5, 4
        assert lib.ppo_collect(h, C.byref(io), 0, fake, 1 << 40, None) == L.PPO_ESHAPE
        io.t_begin = io.t_end = 3
        assert lib.ppo_collect(h, C.byref(io), L.PPO_COLLECT_GRAPH, fake, 16, None) == L.PPO_OK
        io.t_begin, io.t_end = 0, 9
        lens = (C.c_int32 * 4)(8, 6, 7, 1)
        io.lengths = C.cast(lens, L.P_i32)
        assert lib.ppo_collect(h, C.byref(io), L.PPO_COLLECT_TRIM, fake, 1 << 40, None) == L.PPO_ESHAPE
        lens[1], lens[3] = 7, 9
        assert lib.ppo_collect(h, C.byref(io), L.PPO_COLLECT_TRIM, fake, 1 << 40, None) == L.PPO_ESHAPE
        io.N = 0
        assert lib.ppo_collect(h, C.byref(io), 0, fake, 1 << 40, None) == L.PPO_ESHAPE
        assert lib.ppo_collect_graph_count(h) == 0 and lib.ppo_collect_clear(h) == 0
    finally:
        lib.ppo_net_destroy(h)


def test_tile_table_accepts_every_tile_shape_and_rejects_others():
    """The autotuner's table takes tile indices 0..5 and splits 1..256, and
    refuses anything else."""
    lib = L.lib()
    h = C.c_void_p()
    assert lib.ppo_net_create(C.byref(_desc()), C.byref(h)) == L.PPO_OK
    try:
        n = C.c_int(0)
        for tile, split, ok in ((0, 1, True), (5, 256, True), (6, 1, False), (-1, 1, False), (3, 0, False),
                                (3, 257, False)):
            row = (C.c_int64 * 7)(1, 64, 64, 576, 6, tile, split)
            n.value = 1
            st = lib.ppo_autotune_table(h, 1, row, 1, C.byref(n))
            assert (st == L.PPO_OK) == ok, (tile, split)
        assert lib.ppo_autotune_table(h, 0, None, 0, C.byref(n)) == L.PPO_OK and n.value == 1
    finally:
        lib.ppo_net_destroy(h)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.lib()
