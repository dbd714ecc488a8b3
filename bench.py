"""Throughput of one DD-PPO worker on one MI355X.

A step is one full worker iteration (Sec. 3-4): T+1 dependent act steps over
N envs, GAE, then E epochs x M minibatches of (loss backward, Adam).  Frames
per step = sum of the env rollout lengths.  Inputs are seeded synthetic
rollouts (frames U[0,1), goals N(0,1), rewards/dones as in the generator)
staged in device memory before the timed region.  The paper's throughput
procedure (appendix "Additional scaling details") times the last 5 of 10
collect+optimise iterations; --warmup 5 --steps 5 reproduces it.

Prints one JSON line.  The headline value is the bfloat16 form; the float32
form of the same workload is timed beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2500.0     # MI355X dense bf16 MFMA
PEAK_FP32_TFLOPS = 157.3      # MI355X fp32 matrix
PEAK_HBM_GBS = 8000.0
GRAPH = True                  # act loop replayed as one captured HIP graph
AUTOGRAD = False              # update gradient through torch.autograd (C3)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="C2", help="C0..C4 (C2 = bf16 paper-shaped worker)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the float32 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eager", action="store_true", help="launch the act loop eagerly (no HIP graph)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only run a 256 MiB copy and the dominant learner GEMM 3x each (for rocprofv3 --pmc)")
    ap.add_argument("--autograd", choices=["auto", "on", "off"], default="auto",
                    help="take the update's gradient through torch.autograd (auto: for C3)")
    return ap.parse_args()


def stage_env(wl, seed, it, dev):
    """One iteration's environment stream on the device."""
    import torch
    from synth import rollout as R
    ro = R.gen_rollout(wl, seed, it)
    lens = ro["lengths"]
    order = np.argsort(-lens, kind="stable")    # longest first
    obs = ro["obs"][:, order]
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(dev)
    env = {"obs": t(obs).to(torch.bfloat16) if wl.dtype == "bf16" else t(obs),
           "goal": t(ro["goal"][:, order]), "u": t(ro["u"][:, order]),
           "mask": t(ro["mask"][:, order]), "reward": t(ro["reward"][:, order]),
           "done": t(ro["done"][:, order])}
    return env, lens[order]


def _update(w, env, parts, lengths):
    if AUTOGRAD:
        w.update_autograd(env, parts, lengths)
    else:
        w.update(env, parts, lengths)


def run_gpu(wl, steps, warmup, seed, timer=None):
    """timer: (unit, op) whose GEMM kernel launches are timed with HIP events
    over the timed region."""
    import torch
    from paper_1911_00357_amd.worker import PPOHyper, Worker
    from synth import rollout as R
    dev = torch.device("cuda", 0)
    p = wl.ppo
    hp = PPOHyper(p.gamma, p.lam, p.clip, p.value_coef, p.entropy_coef, p.lr, p.epochs, p.minibatches,
                  p.norm_adv)
    w = Worker(wl.net, wl.dtype, wl.T, wl.N, R.init_params(wl.net, seed), hp, dev)
    its = warmup + steps
    envs = [stage_env(wl, seed, i, dev) for i in range(min(its, 2))]
    w.net.autotune(1)             # GEMM tiles tuned during the first warm-up iteration
    parts = R.partitions(wl, seed)
    frames = []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t_start = None
    for i in range(its):
        env, lens = envs[i % len(envs)]
        lengths = None if not wl.ragged else lens
        if i == min(1, warmup):
            w.net.autotune(0)
        if i == warmup:
            torch.cuda.synchronize()
            if timer is not None:
                w.net.gemm_timer_arm(timer[0], timer[1])
            ev[0].record()
            t_start = time.perf_counter()
        w.collect(env, lengths, graph=GRAPH)
        _update(w, env, parts, lengths)
        if i < warmup:
            torch.cuda.synchronize()
            progress(f"warm-up iteration {i + 1}/{warmup} done")
        if i >= warmup:
            frames.append(int(lens.sum()))
    ev[1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    gpu_ms = ev[0].elapsed_time(ev[1])
    timed = None
    if timer is not None:
        timed = w.net.gemm_timer_read()
        w.net.gemm_timer_arm(-1, 0)
    return {"frames": sum(frames), "wall_s": wall, "gpu_ms": gpu_ms, "worker": w, "timed": timed}


def act_update_split(wl, seed):
    """Separate timing of the act phase and the update phase (one iteration)."""
    import torch
    from paper_1911_00357_amd.worker import PPOHyper, Worker
    from synth import rollout as R
    dev = torch.device("cuda", 0)
    p = wl.ppo
    hp = PPOHyper(p.gamma, p.lam, p.clip, p.value_coef, p.entropy_coef, p.lr, p.epochs, p.minibatches)
    w = Worker(wl.net, wl.dtype, wl.T, wl.N, R.init_params(wl.net, seed), hp, dev)
    env, lens = stage_env(wl, seed, 0, dev)
    lengths = None if not wl.ragged else lens
    parts = R.partitions(wl, seed)
    w.net.autotune(1)
    for _ in range(2):
        w.collect(env, lengths, graph=GRAPH)
        _update(w, env, parts, lengths)
        w.net.autotune(0)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    w.collect(env, lengths, graph=GRAPH)
    e[1].record()
    _update(w, env, parts, lengths)
    e[2].record()
    torch.cuda.synchronize()
    return e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), int(lens.sum())


def unpacked_split(wl, seed):
    """The same ragged iteration without packing: one act call per active env
    per step (batch 1) and one learner call per env of each minibatch (each
    followed by its own Adam step is not needed for timing; the per-env calls
    are what packing replaces).  Returns (act ms, update ms, frames)."""
    import torch
    from paper_1911_00357_amd.api import LossCfg
    from paper_1911_00357_amd.worker import PPOHyper, Worker
    from synth import rollout as R
    dev = torch.device("cuda", 0)
    p = wl.ppo
    hp = PPOHyper(p.gamma, p.lam, p.clip, p.value_coef, p.entropy_coef, p.lr, p.epochs, p.minibatches)
    w = Worker(wl.net, wl.dtype, wl.T, wl.N, R.init_params(wl.net, seed), hp, dev)
    env, lens = stage_env(wl, seed, 0, dev)
    parts = R.partitions(wl, seed)
    w.collect(env, lens)
    adv, ret = w.advantages(env, lens)
    ro = w.rollout_view(env, adv, ret)
    cfg = LossCfg(hp.clip, hp.value_coef, hp.entropy_coef)
    scale = w.adam.scale_tensor() if w.bf16 else None

    def act_unpacked():
        for t in range(wl.T + 1):
            for n in range(wl.N):
                if lens[n] < t:
                    break
                # env n's state rows, read and written in place (layer stride N rows)
                H = wl.net.hidden
                row = lambda x: x.reshape(-1)[n * H:]
                out = {"action": w.act_rec[t + 1, n:n + 1], "logp": w.logp[t, n:n + 1],
                       "value": w.value[t, n:n + 1], "h": row(w.h_hist[min(t + 1, wl.T)]),
                       "c": row(w.c_hist[min(t + 1, wl.T)])}
                w.net.act(env["obs"][t, n:n + 1], env["goal"][t, n:n + 1], w.act_rec[t, n:n + 1],
                          env["mask"][t, n:n + 1], row(w.h_hist[t]), row(w.c_hist[t]), env["u"][t, n:n + 1],
                          w.params, w.lp, out=out, state_rows=wl.N)

    def update_unpacked():
        for ep in parts:
            for envs in ep:
                for e in envs:
                    w.net.loss_backward(ro, [int(e)], lens, w.params, w.lp, cfg, loss_scale=scale,
                                        adv_stats=w.adv_stats, grad=w.grad, stats=w.stats)
    act_unpacked()                # warm-up (tiles: the heuristic choice; every env has its own
    update_unpacked()             # frame count, so tuning each one is not part of this comparison)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e[0].record()
    act_unpacked()
    e[1].record()
    update_unpacked()
    e[2].record()
    torch.cuda.synchronize()
    return e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), int(lens.sum())


def cpu_baseline(wl, seed):
    """The FP64 oracle on a bounded sample of the same workload: a 16-step
    rollout of all N envs (17 act steps) and the update over its frames
    (about 10-20 s of host time for the paper-shaped worker)."""
    import oracle
    from synth import rollout as R
    small = wl.with_(T=16)
    flat = R.init_params(wl.net, seed)
    inp = R.gen_rollout(small, seed, 0)
    inp["lengths"] = np.full(small.N, small.T, np.int32)
    h0, c0 = R.gen_state(wl.net, small.N, seed)
    t0 = time.perf_counter()
    rec = oracle.ppo.rollout(flat, wl.net, inp, h0, c0)
    oracle.ppo.update(flat, wl.net, wl.ppo, inp, rec, R.partitions(small, seed))
    dt = time.perf_counter() - t0
    frames = small.T * small.N
    threads = int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", os.cpu_count())))
    return {"value": frames / dt, "unit": "frames/s", "cores": min(threads, os.cpu_count()),
            "kind": "oracle",
            "sample": f"T={small.T} rollout of N={small.N} envs ({small.T + 1} act steps) + {wl.ppo.epochs}x"
                      f"{wl.ppo.minibatches} minibatch updates, {frames} frames, {dt:.1f} s"}


OPS = ["conv forward", "conv data gradient", "conv weight gradient"]


def dominant_gemm(wl, seed, reps=5):
    """The learner's slowest convolution GEMM launch: every trunk unit's
    forward, data-gradient and weight-gradient GEMM at the learner's
    minibatch size, timed with HIP events (selection only).  Returns
    (unit, op, name, per-launch ms table summary)."""
    import torch
    import paper_1911_00357_amd as P
    from paper_1911_00357_amd._lib import PPO_OP_LEARN
    from synth import rollout as R
    dev = torch.device("cuda", 0)
    n = P.Net(wl.net, wl.dtype)
    params = torch.tensor(R.init_params(wl.net, seed), device=dev)
    lp = P.cast_bf16(params) if wl.dtype == "bf16" else None
    grad = torch.zeros_like(params)
    F = wl.T * wl.N // wl.ppo.minibatches
    nunits = n.probe(PPO_OP_LEARN, F, 1, 3)[3][0]
    n.autotune(1)                 # each problem is tuned on its first (untimed) launch
    rows = []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for u in range(nunits):
        name = n.probe(PPO_OP_LEARN, F, 1, 0, u)[0]
        for op in (0, 1, 2):
            if op == 1 and u == 0:
                continue              # the first convolution needs no data gradient
            n.bench_unit_gemm(op, u, F, params, lp, grad, 1)
            ev[0].record()
            fl = n.bench_unit_gemm(op, u, F, params, lp, grad, reps)
            ev[1].record()
            torch.cuda.synchronize()
            rows.append((ev[0].elapsed_time(ev[1]) / reps, fl, name, op, u))
    t_ms, fl, name, op, u = max(rows)
    tot_t = sum(r[0] for r in rows)
    tot_f = sum(r[1] for r in rows)
    del n, params, lp, grad
    torch.cuda.empty_cache()
    return u, op, name, round(tot_f / (tot_t / 1e3) / 1e12, 3)


def committed_gemm(wl):
    """(unit, op, name, None) of the roofline kernel named in the committed
    bench line of this workload (profiles/bench_<workload>.json)."""
    import paper_1911_00357_amd as P
    from paper_1911_00357_amd._lib import PPO_OP_LEARN
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", f"bench_{wl.name}.json")
    with open(path) as f:
        label = json.load(f)["roofline"]["kernel"]
    op = next(i for i, s in enumerate(OPS) if label.startswith(s + " GEMM of "))
    name = label[len(OPS[op] + " GEMM of "):]
    n = P.Net(wl.net, wl.dtype)
    F = wl.T * wl.N // wl.ppo.minibatches
    for u in range(n.probe(PPO_OP_LEARN, F, 1, 3)[3][0]):
        if n.probe(PPO_OP_LEARN, F, 1, 0, u)[0] == name:
            return u, op, name, None
    raise SystemExit(f"unit {name} not found")


COPY_BYTES = 256 << 20


def pmc_probe(wl, seed, sel):
    """Calibration copy (COPY_BYTES read + written per launch) and the dominant
    learner GEMM, three launches each, for HBM byte counters."""
    import torch
    import paper_1911_00357_amd as P
    from synth import rollout as R
    dev = torch.device("cuda", 0)
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    n = P.Net(wl.net, wl.dtype)
    params = torch.tensor(R.init_params(wl.net, seed), device=dev)
    lp = P.cast_bf16(params) if wl.dtype == "bf16" else None
    grad = torch.zeros_like(params)
    F = wl.T * wl.N // wl.ppo.minibatches
    n.autotune(1)
    n.bench_unit_gemm(sel[1], sel[0], F, params, lp, grad, 1)   # tunes the problem as the worker does
    n.autotune(0)
    torch.cuda.synchronize()
    n.bench_unit_gemm(sel[1], sel[0], F, params, lp, grad, 3)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": {"copy_bytes": COPY_BYTES, "kernel": f"{OPS[sel[1]]} GEMM of {sel[2]}",
                                    "frames": F}}), flush=True)


def traffic_bytes(kernel, workload):
    """Per-launch HBM bytes (fetch + write) of `kernel` from the committed PMC
    summary, or None when that summary is missing, was taken on another
    workload or on other GEMM sources than the ones built now."""
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for name in rec.get("sources", []):
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), name), "rb") as f:
            h.update(f.read())
    if rec.get("kernel") != kernel or rec.get("workload") != workload or rec.get("sources_sha256") != h.hexdigest():
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def roofline_live(wl, sel, timed):
    """Roofline entry of the dominant GEMM kernel from its launches inside the
    timed steps (HIP events on the learner's stream around the kernel
    itself): achieved = summed 2*M*N*K / summed duration."""
    u, op, name, all_tf = sel
    launches, ms, fl = timed
    peak = PEAK_BF16_TFLOPS if wl.dtype == "bf16" else PEAK_FP32_TFLOPS
    if launches == 0 or ms <= 0:
        return {"bound": "mfma", "achieved": None, "peak": peak, "unit": "TFLOP/s", "frac": None,
                "traffic": None, "kernel": f"{OPS[op]} GEMM of {name}"}
    ach = fl / (ms / 1e3) / 1e12
    return {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 5), "traffic": traffic_bytes(f"{OPS[op]} GEMM of {name}", wl.name),
            "kernel": f"{OPS[op]} GEMM of {name}", "launches": launches,
            "avg_launch_us": round(ms / launches * 1e3, 2), "flops_per_launch": fl / launches,
            "all_conv_gemms_tflops_microbench": all_tf}


def flops_per_frame(net):
    """Forward multiply-adds x2 of the encoder convolutions, the visual FC and
    the LSTM/head GEMMs for one frame."""
    from synth.layout import tensor_list
    hw = net.enc_hw
    f = 0
    if net.trunk == "tiny":
        h1 = hw // 2
        h2 = h1 // 2
        f += 2 * h1 * h1 * net.tiny_ch[0] * 9 * net.in_ch + 2 * h2 * h2 * net.tiny_ch[1] * 9 * net.tiny_ch[0]
    else:
        h = hw // 2
        f += 2 * h * h * net.base_width * 49 * net.in_ch
        h //= 2
        cin = net.base_width
        for s, nb in enumerate(net.blocks):
            w = net.base_width << s
            for j in range(nb):
                st = 2 if (j == 0 and s > 0) else 1
                ho = h // st
                f += 2 * h * h * w * cin + 2 * ho * ho * w * 9 * w + 2 * ho * ho * 4 * w * w
                if j == 0:
                    f += 2 * ho * ho * 4 * w * cin
                cin = 4 * w
                h = ho
        f += 2 * h * h * net.compress_ch * 9 * cin
    f += 2 * net.flat_dim * net.vis_hidden
    H = net.hidden
    f += 2 * 4 * H * (net.lstm_in + H) + (net.lstm_layers - 1) * 2 * 4 * H * 2 * H
    f += 2 * (net.num_actions + 1) * H
    return f


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    a = parse()
    global GRAPH, AUTOGRAD
    GRAPH = not a.eager
    AUTOGRAD = a.autograd == "on" or (a.autograd == "auto" and a.workload == "C3")
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; the gradient all-reduce of a "
                                   "multi-GPU worker group is not implemented", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    from synth.configs import WORKLOADS
    wl = WORKLOADS[a.workload]
    if a.pmc_probe:
        # the kernel the committed bench line names (counter runs distort the timing-based selection)
        pmc_probe(wl, a.seed, committed_gemm(wl))
        return
    progress(f"workload {a.workload}: selecting the dominant learner GEMM")
    sel = dominant_gemm(wl, a.seed)
    progress("timed run")
    res = run_gpu(wl, a.steps, a.warmup, a.seed, timer=sel[:2])
    roof = roofline_live(wl, sel, res["timed"])
    fps = res["frames"] / (res["gpu_ms"] / 1e3)
    ms_step = res["gpu_ms"] / a.steps
    frames_step = res["frames"] / a.steps
    out = {"metric": "PPO act+update frames/s", "value": round(fps, 2), "unit": "frames/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16" if wl.dtype == "bf16" else "f32", "data": "synthetic",
           "config": {"workload": wl.name, "T": wl.T, "N": wl.N, "frame": f"{wl.net.in_ch}x{wl.net.in_hw}x{wl.net.in_hw}",
                      "encoder": "resnet50 halved widths, GroupNorm" if wl.net.trunk == "resnet" else "tiny",
                      "lstm": f"{wl.net.lstm_layers}x{wl.net.hidden}", "epochs": wl.ppo.epochs,
                      "minibatches": wl.ppo.minibatches, "frames_per_step": frames_step,
                      "parallelism": "single worker",
                      "gradient": "torch.autograd.Function, activations recomputed" if AUTOGRAD
                      else "ppo_loss_backward", "gemm_tiles": "autotuned in warm-up"},
           "wall_s": round(res["wall_s"], 3)}
    del res
    torch.cuda.empty_cache()
    progress("act / update split")
    act_ms, upd_ms, fr = act_update_split(wl, a.seed)
    out["act_ms"], out["update_ms"] = round(act_ms, 3), round(upd_ms, 3)
    out["act_frames_per_s"] = round((fr + wl.N) / (act_ms / 1e3), 1)
    out["update_frames_per_s"] = round(fr / (upd_ms / 1e3), 1)
    fpf = flops_per_frame(wl.net)
    upd_flops = 3 * fpf * fr * wl.ppo.epochs
    peak = PEAK_BF16_TFLOPS if wl.dtype == "bf16" else PEAK_FP32_TFLOPS
    # whole iteration: act forward of every frame (+ the bootstrap step) and E x (forward + backward)
    step_flops = fpf * ((1 + 3 * wl.ppo.epochs) * frames_step + wl.N)
    out["step_tflops"] = round(step_flops / (ms_step / 1e3) / 1e12, 3)
    out["step_mfma_frac"] = round(step_flops / (ms_step / 1e3) / 1e12 / (PEAK_BF16_TFLOPS if wl.dtype == "bf16" else PEAK_FP32_TFLOPS), 5)
    out["update_tflops"] = round(upd_flops / (upd_ms / 1e3) / 1e12, 3)
    out["update_mfma_frac"] = round(upd_flops / (upd_ms / 1e3) / 1e12 / peak, 5)
    if wl.dtype == "bf16" and not a.no_fp32:
        torch.cuda.empty_cache()
        progress("float32 form")
        wl32 = wl.with_(dtype="f32")
        r32 = run_gpu(wl32, a.steps, 1, a.seed)
        out["fp32_value"] = round(r32["frames"] / (r32["gpu_ms"] / 1e3), 2)
        out["bf16_speedup_vs_fp32"] = round(out["value"] / out["fp32_value"], 3)
        del r32
    if wl.ragged:
        torch.cuda.empty_cache()
        progress("unpacked per-env launches")
        ua, uu, ufr = unpacked_split(wl, a.seed)
        out["unpacked_act_frames_per_s"] = round((ufr + wl.N) / (ua / 1e3), 1)
        out["unpacked_update_frames_per_s"] = round(ufr / (uu / 1e3), 1)
        out["packed_speedup_act"] = round(out["act_frames_per_s"] / out["unpacked_act_frames_per_s"], 3)
        out["packed_speedup_update"] = round(out["update_frames_per_s"] / out["unpacked_update_frames_per_s"], 3)
        out["unpacked_gemm_tiles"] = "heuristic"
    out["roofline"] = roof
    if not a.no_cpu:
        progress("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(wl, a.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
