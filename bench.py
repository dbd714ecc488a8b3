"""Throughput of one DD-PPO worker on one MI355X.

A step is one full worker iteration (Sec. 3-4): T+1 dependent act steps over
N envs, GAE, then E epochs x M minibatches of (loss backward, Adam).  Frames
per step = sum of the env rollout lengths.  Inputs are seeded synthetic
rollouts (frames U[0,1), goals N(0,1), rewards/dones as in the generator)
staged in device memory before the timed region.

Protocol (appendix "Additional scaling details": 10 seeds, throughput over
the last iterations, bootstrapped 95% confidence interval): for each seed,
--warmup untimed iterations, then --steps timed iterations; the headline
value is the median over seeds of frames / timed GPU time, with a bootstrap
95% interval of that median.  The float32 form of the same workload is timed
on the same seeds.

Prints one JSON line.  The roofline entry is the act step's convolution
GEMMs (the largest kernel class by time), timed live with HIP events right
after the timed iterations (each unit's product as the act graph runs it,
many launches back to back); the learner's slowest convolution GEMM is a
second entry.  The CPU baseline is
the float64 oracle on a bounded sample of the same workload, with the GPU's
per-output errors on that sample.
"""
from __future__ import annotations

import argparse
import gc
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
ACT_REPS = 64                 # back-to-back launches per act product in the roofline timing


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seeds", type=int, default=10, help="seeds 0..S-1 (median and bootstrap 95%% CI)")
    ap.add_argument("--workload", default="C2", help="C0..C6 (C2 = bf16 paper-shaped worker; C5, C6 the "
                                                     "SE-ResNeXt50 and SE-ResNeXt101 + 1024-d LSTM agents)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the float32 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--eager", action="store_true", help="launch the act loop eagerly (no HIP graph)")
    ap.add_argument("--pmc-probe", choices=["act", "learner"],
                    help="only run a 256 MiB copy and then every convolution GEMM at the act or the "
                         "learner batch (for rocprofv3 --pmc)")
    ap.add_argument("--tiles-out", help="write the tuned tile table (JSON) of the timed form here")
    ap.add_argument("--tiles-in", help="use this tile table (from --tiles-out) instead of tuning")
    ap.add_argument("--autograd", choices=["auto", "on", "off"], default="auto",
                    help="take the update's gradient through torch.autograd (auto: for C3)")
    return ap.parse_args()


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def trace_marker():
    """A one-block bfloat16 cast of three values: a dispatch no other step of
    the bench makes (parameter casts cover whole vectors), so a kernel trace
    can find the phases it separates.  Synchronises."""
    import torch
    import paper_1911_00357_amd as P
    P.cast_bf16(torch.zeros(3, device="cuda"))
    torch.cuda.synchronize()


def stage_env(wl, seed, it, dev):
    """One iteration's environment stream on the device (envs longest first)."""
    import torch
    from synth import rollout as R
    ro = R.gen_rollout(wl, seed, it)
    lens = ro["lengths"]
    order = np.argsort(-lens, kind="stable")
    obs = ro["obs"][:, order]
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(dev)
    env = {"obs": t(obs).to(torch.bfloat16) if wl.dtype == "bf16" else t(obs),
           "goal": t(ro["goal"][:, order]), "u": t(ro["u"][:, order]),
           "mask": t(ro["mask"][:, order]), "reward": t(ro["reward"][:, order]),
           "done": t(ro["done"][:, order])}
    return env, lens[order]


def _hyper(wl):
    from paper_1911_00357_amd.worker import PPOHyper
    p = wl.ppo
    return PPOHyper(p.gamma, p.lam, p.clip, p.value_coef, p.entropy_coef, p.lr, p.epochs, p.minibatches,
                    p.norm_adv)


def _update(w, env, parts, lengths):
    if AUTOGRAD:
        w.update_autograd(env, parts, lengths)
    else:
        w.update(env, parts, lengths)


def run_seed(wl, seed, steps, warmup, net=None, act_timer=True):
    """Warm-up and timed iterations of one seed; with act_timer, then the act
    step's convolution products timed (act_gemms_live; the runtime that comes
    with torch refuses event nodes inside the captured graph itself).
    Returns frames, GPU ms, wall s, the act-GEMM timing and the worker."""
    import torch
    from paper_1911_00357_amd.worker import Worker
    from synth import rollout as R
    dev = torch.device("cuda", 0)
    w = Worker(wl.net, wl.dtype, wl.T, wl.N, R.init_params(wl.net, seed), _hyper(wl), dev, net=net)
    its = warmup + steps
    envs = [stage_env(wl, seed, i, dev) for i in range(min(its, 2))]
    parts = R.partitions(wl, seed)
    frames = 0
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t_start = None
    for i in range(its):
        env, lens = envs[i % len(envs)]
        lengths = None if not wl.ragged else lens
        if i == warmup:
            if act_timer:
                trace_marker()          # kernel-trace landmark: the timed iterations start
            torch.cuda.synchronize()
            ev[0].record()
            t_start = time.perf_counter()
        w.collect(env, lengths, graph=GRAPH, trim=wl.ragged)
        _update(w, env, parts, lengths)
        if i < warmup:
            torch.cuda.synchronize()
        else:
            frames += int(lens.sum())
    ev[1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    # run health, read after the timed region: Adam's skipped steps (a non-finite
    # gradient), the last minibatch's loss statistics, the recurrence's barrier status
    st = w.adam.state()
    health = {"adam_steps": int(st["step"]), "adam_skipped": int(st["skipped"]), "loss_scale": float(st["scale"]),
              "loss_finite": bool(torch.isfinite(w.stats).all()), "recurrence_failed": bool(w.net.recurrence_failed())}
    act = act_gemms_live(w, wl) if act_timer else None
    return {"frames": frames, "gpu_ms": ev[0].elapsed_time(ev[1]), "wall_s": wall, "act": act, "worker": w,
            "health": health}


def act_gemms_live(w, wl, reps=ACT_REPS):
    """The act step's convolution products timed live: each trunk unit's
    product as ppo_act runs it at the act batch (same tiles and K split, from
    the table tuned in the warm-up), `reps` launches back to back between
    two HIP events on the stream they run on.  Returns (launches, ms, FLOPs,
    weight bytes, per-unit us)."""
    import torch
    from paper_1911_00357_amd._lib import PPO_OP_LEARN
    trace_marker()                      # kernel-trace landmark: the timed act products follow
    n = w.net
    N = wl.N
    nunits = n.probe(PPO_OP_LEARN, N, 1, 3)[3][0]
    wcount = {name: cnt for name, _, cnt in n.tensors()}
    esize = 2 if wl.dtype == "bf16" else 4
    grad = torch.zeros_like(w.params)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    tot_ms = tot_fl = tot_b = 0.0
    per = []
    for u in range(nunits):
        name = n.probe(PPO_OP_LEARN, N, 1, 0, u)[0]
        n.bench_unit_gemm(3, u, N, w.params, w.lp, grad, 1)
        ev[0].record()
        fl = n.bench_unit_gemm(3, u, N, w.params, w.lp, grad, reps)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        tot_ms += ms
        tot_fl += fl * reps
        tot_b += wcount[name] * esize * reps
        per.append((name, round(ms / reps * 1e3, 3)))
    return nunits * reps, tot_ms, tot_fl, tot_b, per


def run_seeds(wl, seeds, steps, warmup, label, tiles=None):
    """Every seed on one shared library handle (its tile table is tuned in the
    first seed's first warm-up iteration, or loaded from `tiles`).  Returns
    per-seed results (without workers) and the first seed's worker."""
    import torch
    import paper_1911_00357_amd as P
    net = P.Net(wl.net, wl.dtype)
    if tiles:
        net.tile_table(tiles)
    else:
        net.autotune(1)
    out, first = [], None
    for k, seed in enumerate(seeds):
        r = run_seed(wl, seed, steps, warmup, net=net, act_timer=(k == 0))
        if k == 0:
            net.autotune(0)
            first = r.pop("worker")
        else:
            r.pop("worker").release()
        out.append(r)
        progress(f"{label} seed {seed}: {r['frames'] / (r['gpu_ms'] / 1e3):.1f} frames/s")
        gc.collect()
        torch.cuda.empty_cache()
    return out, first


def encoder_label(net):
    if net.trunk == "tiny":
        return "tiny"
    depth = {(3, 4, 6, 3): "50", (3, 4, 23, 3): "101"}.get(tuple(net.blocks), str(tuple(net.blocks)))
    if net.trunk == "seresnext":
        return (f"se-resnext{depth} halved widths ({net.cardinality} groups, squeeze-excite 1/"
                f"{net.se_reduction}), GroupNorm")
    return f"resnet{depth} halved widths, GroupNorm"


def median_ci(x, n_boot=10000, seed=0):
    """Median of x and a bootstrap 95% interval of the median (percentile)."""
    x = np.asarray(x, np.float64)
    if x.size == 1:
        return float(x[0]), [float(x[0]), float(x[0])]
    g = np.random.default_rng(seed)
    meds = np.median(x[g.integers(0, x.size, (n_boot, x.size))], axis=1)
    return float(np.median(x)), [float(np.percentile(meds, 2.5)), float(np.percentile(meds, 97.5))]


def act_update_split(wl, seed, net):
    """Separate timing of the act phase and the update phase (one iteration)."""
    import torch
    from paper_1911_00357_amd.worker import Worker
    from synth import rollout as R
    dev = torch.device("cuda", 0)
    w = Worker(wl.net, wl.dtype, wl.T, wl.N, R.init_params(wl.net, seed), _hyper(wl), dev, net=net)
    env, lens = stage_env(wl, seed, 0, dev)
    lengths = None if not wl.ragged else lens
    parts = R.partitions(wl, seed)
    for _ in range(2):
        w.collect(env, lengths, graph=GRAPH, trim=wl.ragged)
        _update(w, env, parts, lengths)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    w.collect(env, lengths, graph=GRAPH, trim=wl.ragged)
    e[1].record()
    _update(w, env, parts, lengths)
    e[2].record()
    torch.cuda.synchronize()
    w.release()
    return e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), int(lens.sum())


def unpacked_split(wl, seed):
    """The same ragged iteration without packing: one act call per active env
    per step (batch 1) and one learner call per env of each minibatch (the
    per-env calls are what packing replaces).  Returns (act ms, update ms,
    frames)."""
    import torch
    from paper_1911_00357_amd.api import LossCfg
    from paper_1911_00357_amd.worker import Worker
    from synth import rollout as R
    dev = torch.device("cuda", 0)
    hp = _hyper(wl)
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
    act_unpacked()                # warm-up (tiles: the heuristic choice)
    update_unpacked()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e[0].record()
    act_unpacked()
    e[1].record()
    update_unpacked()
    e[2].record()
    torch.cuda.synchronize()
    w.release()
    return e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), int(lens.sum())


# --------------------------------------------------------------- CPU baseline
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def blas_threads():
    from threadpoolctl import threadpool_info
    n = [i["num_threads"] for i in threadpool_info() if i.get("user_api") == "blas"]
    return max(n) if n else 1


def gpu_sample(wl, small, seed, inp, parts):
    """The GPU worker on the oracle's sample: rollout outputs, advantages and
    the first minibatch's loss statistics, gradient (unscaled) and the
    decisions it took (ReLU patterns, max-pool winners; bfloat16 operand
    codes), read from the workspace as the parity tests do."""
    from tests.test_gpu_parity import gpu_decisions
    import torch
    from paper_1911_00357_amd.worker import Worker
    from synth import rollout as R
    dev = torch.device("cuda", 0)
    w = Worker(wl.net, wl.dtype, small.T, small.N, R.init_params(wl.net, seed), _hyper(small), dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(dev)
    env = {k: t(inp[k]) for k in ("goal", "u", "mask", "reward", "done")}
    env["obs"] = t(inp["obs"]).to(torch.bfloat16) if wl.dtype == "bf16" else t(inp["obs"])
    w.collect(env)
    first = {}

    def hook(wk):
        if not first:
            S = wk.adam.state()["scale"] if wk.bf16 else 1.0
            first["grad"] = wk.grad.cpu().numpy().astype(np.float64) / S
            first["stats"] = wk.stats.cpu().numpy().astype(np.float64)
            B = len(parts[0][0])
            first["decisions"] = gpu_decisions(wk.net, wl.net, small.T * B, B,
                                               {"action": np.zeros((small.T, B)), "lens": np.full(B, small.T)},
                                               codes=wk.bf16)
    adv, ret = w.update(env, parts, on_minibatch=hook)
    out = {"action": w.act_rec[1:].cpu().numpy(), "value": w.value.cpu().numpy().astype(np.float64),
           "logp": w.logp.cpu().numpy().astype(np.float64), "adv": adv.cpu().numpy().astype(np.float64),
           "ret": ret.cpu().numpy().astype(np.float64), **first}
    w.release()
    return out


def cpu_baseline(wl, seed):
    """The float64 oracle on a bounded sample of the same workload: a 16-step
    rollout of all N envs (17 act steps) and the update over its frames,
    timed with the host's BLAS threads (about 10-20 s for the paper-shaped
    worker), and a 2-step sample with one thread.  The GPU's bfloat16 and
    float32 forms are run on the same sample (the GPU's sampled actions fed
    to the oracle as previous actions) and their per-output errors against
    the oracle reported: values, log-probs, advantages, returns, the first
    minibatch's loss and gradient (the GPU's ReLU / max-pool decisions, and in
    bfloat16 its operand codes, imposed on the oracle as in the parity tests:
    exact float64 reference, and for bfloat16 also the precision form)."""
    from threadpoolctl import threadpool_limits
    import oracle
    from oracle import nn as onn
    from synth import rollout as R

    def rel(x, ref):
        x, ref = np.asarray(x, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
        return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-30))

    def sample(T):
        small = wl.with_(T=T)
        inp = R.gen_rollout(small, seed, 0)
        inp["lengths"] = np.full(small.N, small.T, np.int32)
        return small, inp, R.partitions(small, seed)

    flat = R.init_params(wl.net, seed)
    small, inp, parts = sample(16)
    h0, c0 = R.gen_state(wl.net, small.N, seed)
    gpu = {dt: gpu_sample(wl.with_(dtype=dt), small, seed, inp, parts) for dt in ("bf16", "f32")}
    act = gpu["f32"]["action"]
    threads = blas_threads()
    t0 = time.perf_counter()
    rec = oracle.ppo.rollout(flat, wl.net, inp, h0, c0, forced_actions=act)
    lp = np.take_along_axis(onn.log_softmax(rec["logits"]), act[..., None], axis=2)[..., 0]
    rec["action"], rec["logp"] = act, lp
    upd = oracle.ppo.update(flat, wl.net, wl.ppo, inp, rec, parts)
    dt = time.perf_counter() - t0
    frames = small.T * small.N
    # the first minibatch again, with each side's decisions made the same way (the GPU's, each
    # checked to sit at a near-kink or rounding midpoint, as in the parity tests)
    from tests.gpu_util import tensor_errors
    from tests.test_gpu_parity import LossCase, oracle_refs
    mb = oracle.ppo.minibatch_inputs(wl.net, inp, rec, upd["adv"], upd["ret"], np.asarray(parts[0][0]))
    errors = {}
    for k, g in gpu.items():
        c = LossCase()
        c.g, c.s = g["grad"], g["stats"]
        coded = g["decisions"]
        dec = {kk: v for kk, v in coded.items() if not kk.startswith("q:")}
        oracle_refs(c, wl.net, k, flat, mb, dec, coded=coded if k == "bf16" else None)
        s_ref = c.s_exact
        te = tensor_errors(wl.net, c.g, c.g_exact)
        worst = max(te, key=lambda kk: te[kk][0])
        errors[k] = {"values": rel(g["value"], rec["value"]), "log_probs": rel(g["logp"], lp),
                     "advantages": rel(g["adv"], upd["adv"]), "returns": rel(g["ret"], upd["ret"]),
                     "loss": abs(g["stats"][0] - s_ref[0]) /
                             (abs(s_ref[1]) + wl.ppo.value_coef * abs(s_ref[2]) + wl.ppo.entropy_coef * abs(s_ref[3])),
                     "gradient": rel(c.g, c.g_exact), "gradient_worst_tensor": [worst, round(te[worst][0], 8)],
                     "decisions_flipped": int(sum(f for _, f in c.flips.values())),
                     "actions_differing": int((g["action"] != act).sum())}
        if k == "bf16":
            tf = tensor_errors(wl.net, c.g, c.g_form)
            errors[k]["gradient_vs_bf16_form"] = rel(c.g, c.g_form)
            errors[k]["gradient_vs_bf16_form_worst_tensor"] = round(max(v[0] for v in tf.values()), 8)
            errors[k]["bf16_form_gradient_vs_exact"] = rel(c.g_own, c.g_exact)
        errors[k] = {kk: (round(v, 8) if isinstance(v, float) else v) for kk, v in errors[k].items()}
    small1, inp1, parts1 = sample(2)
    with threadpool_limits(1):
        t1 = time.perf_counter()
        rec1 = oracle.ppo.rollout(flat, wl.net, inp1, *R.gen_state(wl.net, small1.N, seed))
        oracle.ppo.update(flat, wl.net, wl.ppo, inp1, rec1, parts1)
        dt1 = time.perf_counter() - t1
    return {"value": frames / dt, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"T={small.T} rollout of N={small.N} envs ({small.T + 1} act steps) + {wl.ppo.epochs}x"
                      f"{wl.ppo.minibatches} minibatch updates, {frames} frames, {dt:.1f} s",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "one_thread": {"value": small1.T * small1.N / dt1, "unit": "frames/s",
                           "sample": f"T={small1.T} rollout of N={small1.N} envs + the same update, "
                                     f"{small1.T * small1.N} frames, {dt1:.1f} s"},
            "gpu_errors_vs_oracle": errors}


# ------------------------------------------------------------------ roofline
OPS = ["conv forward", "conv data gradient", "conv weight gradient"]
ACT_KERNEL = "act-step convolution GEMMs (gemm_kernel<ConvFwdProb<bf16>, ...>, all tiles)"


def dominant_gemm(wl, seed, reps=5):
    """The learner's slowest convolution GEMM launch: every trunk unit's
    forward, data-gradient and weight-gradient GEMM at the learner's
    minibatch size, timed with HIP events (selection only).  Returns
    (unit, op, name, aggregate TFLOP/s of all of them)."""
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


def learner_gemm_live(w, wl, env, parts, sel):
    """The dominant learner GEMM timed with HIP events on the learner's
    stream around the kernel itself, over one update."""
    import torch
    u, op, name, all_tf = sel
    w.net.gemm_timer_arm(u, op)
    _update(w, env, parts, None)
    torch.cuda.synchronize()
    launches, ms, fl, _ = w.net.gemm_timer_read()
    w.net.gemm_timer_arm(-1, 0)
    peak = PEAK_BF16_TFLOPS if wl.dtype == "bf16" else PEAK_FP32_TFLOPS
    if launches == 0 or ms <= 0:
        return {"bound": "mfma", "achieved": None, "peak": peak, "unit": "TFLOP/s", "frac": None,
                "kernel": f"{OPS[op]} GEMM of {name}"}
    ach = fl / (ms / 1e3) / 1e12
    return {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 5), "kernel": f"{OPS[op]} GEMM of {name}", "launches": launches,
            "avg_launch_us": round(ms / launches * 1e3, 2), "flops_per_launch": fl / launches,
            "all_conv_gemms_tflops_microbench": all_tf}


def traffic_bytes(kernel, workload):
    """Per-launch HBM bytes (fetch + write) of `kernel` from the committed
    counter summary, or None when it is missing, was taken on another
    workload or on other GEMM sources than the ones built now."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        recs = json.load(f)
    for rec in recs if isinstance(recs, list) else [recs]:
        h = hashlib.sha256()
        for name in rec.get("sources", []):
            with open(os.path.join(ROOT, name), "rb") as f:
                h.update(f.read())
        if rec.get("kernel") == kernel and rec.get("workload") == workload and \
                rec.get("sources_sha256") == h.hexdigest():
            return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return None


def act_roofline(wl, act):
    """Roofline entry of the act step's convolution GEMMs from their HIP-event
    durations: algorithmic bytes = the weight operand
    of each product (every activation of an act step could stay on chip), the
    bound of a batch-4 product; the matrix-core fraction of the same launches
    is given beside it."""
    launches, ms, fl, wb, per = act
    if not launches or ms <= 0:
        return {"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
                "traffic": None, "kernel": ACT_KERNEL}
    ach = wb / (ms / 1e3) / 1e9
    peak_mfma = PEAK_BF16_TFLOPS if wl.dtype == "bf16" else PEAK_FP32_TFLOPS
    tflops = fl / (ms / 1e3) / 1e12
    tr = traffic_bytes(ACT_KERNEL, wl.name)
    return {"bound": "hbm", "achieved": round(ach, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 6), "traffic": tr, "kernel": ACT_KERNEL,
            "launches": launches, "reps_per_unit": ACT_REPS, "avg_launch_us": round(ms / launches * 1e3, 3),
            "bytes_per_launch": wb / launches, "flops_per_launch": fl / launches,
            "mfma_tflops": round(tflops, 3), "mfma_frac": round(tflops / peak_mfma, 6),
            "timed": f"after the timed iterations: each unit's act product (the tiles and K split the "
                     f"graph replays) launched {ACT_REPS} times back to back between two HIP events",
            "per_unit_us": per}


def flops_per_frame(net):
    """Forward multiply-adds x2 of the encoder convolutions, the visual FC and
    the LSTM/head GEMMs for one frame."""
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


# ------------------------------------------------------------------ counters
COPY_BYTES = 256 << 20




def pmc_probe(wl, seed, what, tiles=None):
    """Calibration copy (COPY_BYTES read + written per launch, three launches),
    then, after a landmark, every trunk unit's convolution GEMMs launched once
    through ppo_bench_unit_gemm, tiles tuned first as the worker tunes them
    (or taken from a tile table the benchmark wrote): 'act' the forward
    products as the act step runs them (N frames, split-K partials left for
    the GroupNorm), 'learner' the forward, data-gradient and weight-gradient
    products at the learner's minibatch size.  For HBM-byte and matrix-core
    counters per dispatch (no other kernel runs between the landmark and the
    end)."""
    import torch
    import paper_1911_00357_amd as P
    from paper_1911_00357_amd._lib import PPO_OP_LEARN
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
    F = wl.N if what == "act" else wl.T * wl.N // wl.ppo.minibatches
    ops = (3,) if what == "act" else (0, 1, 2)
    nunits = n.probe(PPO_OP_LEARN, F, 1, 3)[3][0]
    todo = [(op, u) for u in range(nunits) for op in ops if not (op == 1 and u == 0)]
    if tiles:
        n.tile_table(tiles)
    n.autotune(0 if tiles else 1)
    for op, u in todo:
        n.bench_unit_gemm(op, u, F, params, lp, grad, 1)
    n.autotune(0)
    trace_marker()
    for op, u in todo:
        n.bench_unit_gemm(op, u, F, params, lp, grad, 1)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": {"copy_bytes": COPY_BYTES, "what": what, "frames": F, "launches": len(todo)}}),
          flush=True)


# ------------------------------------------------------- profile summaries
def _is_marker(r):
    return r["Kernel_Name"].startswith("cast_bf16_kernel") and int(r.get("Grid_Size_X", r.get("Grid_Size", 0))) <= 256


def _short(n):
    n = n.replace("(anonymous namespace)::", "")
    return n.split("(")[0].replace("unsigned short", "bf16")[:110]


def summarize_trace(csv_path, log_path=None, ref_path=None):
    """Markdown summary of a kernel trace of this benchmark: the timed
    iteration (between the first two landmarks) split into act loop and
    update at its GAE launch, and the act convolution GEMMs the benchmark
    times after the second landmark, beside the benchmark line of the same
    run (log_path) and of an unprofiled run with the same tiles (ref_path)."""
    import collections
    import csv
    rows = sorted(csv.DictReader(open(csv_path)), key=lambda r: int(r["Start_Timestamp"]))
    dur = lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0
    marks = [i for i, r in enumerate(rows) if _is_marker(r)]
    out = []

    def table(sub, title, top=25):
        busy = sum(dur(r) for r in sub)
        span = (int(sub[-1]["End_Timestamp"]) - int(sub[0]["Start_Timestamp"])) / 1000.0
        g = collections.defaultdict(lambda: [0, 0.0])
        for r in sub:
            x = g[_short(r["Kernel_Name"])]
            x[0] += 1
            x[1] += dur(r)
        out.append(f"\n## {title}: {len(sub)} dispatches, span {span / 1000:.2f} ms, kernel busy {busy / 1000:.2f} ms\n")
        out.append("| calls | total ms | avg us | % | kernel |\n|---:|---:|---:|---:|---|")
        for k, (n, t) in sorted(g.items(), key=lambda kv: -kv[1][1])[:top]:
            out.append(f"| {n} | {t / 1000:.2f} | {t / n:.2f} | {100 * t / busy:.1f} | `{k}` |")

    if len(marks) >= 2:
        timed = rows[marks[0] + 1:marks[1]]
        gae = next(i for i, r in enumerate(timed) if r["Kernel_Name"].startswith("gae_kernel"))
        table(timed[:gae], "act loop of the timed iteration (129 act steps, one graph replay)")
        conv = [dur(r) for r in timed[:gae] if "ConvFwdProb" in r["Kernel_Name"]]
        out.append(f"\nact convolution GEMMs in the graph replay: {len(conv)} launches, average "
                   f"{sum(conv) / max(len(conv), 1):.3f} us")
        out.extend(act_step_positions(timed[:gae], dur))
        table(timed[gae:], "update of the timed iteration")
        after = [r for r in rows[marks[1] + 1:] if "ConvFwdProb" in r["Kernel_Name"]]
        line = None
        if log_path:
            for l in open(log_path):
                if l.startswith("{") and '"roofline"' in l:
                    line = json.loads(l)["roofline"]
        n = line["launches"] if line else 0
        reps = line.get("reps_per_unit", 0) if line else 0
        # per unit: one untimed launch, then `reps` between the events
        leg = [r for i, r in enumerate(after[:n + n // max(reps, 1)]) if reps and i % (reps + 1)]
        if leg:
            avg = sum(dur(r) for r in leg) / len(leg)
            units = [leg[i:i + reps] for i in range(0, len(leg), reps)]
            span = sum((int(u[-1]["End_Timestamp"]) - int(u[0]["Start_Timestamp"])) / 1000.0 for u in units)
            per_span = span / len(leg)
            out.append(f"\n## roofline kernel: {line['kernel']}\n\n"
                       f"The act products the benchmark times after the second landmark: {len(leg)} launches "
                       f"({len(units)} units x {reps}), trace average duration {avg:.3f} us, first-to-last span "
                       f"per launch {per_span:.3f} us; {line['bytes_per_launch']:.0f} algorithmic bytes and "
                       f"{line['flops_per_launch']:.0f} FLOP per launch, i.e. "
                       f"{line['bytes_per_launch'] / avg / 1e3:.2f} GB/s "
                       f"({line['bytes_per_launch'] / avg / 1e3 / PEAK_HBM_GBS:.6f} of {PEAK_HBM_GBS:.0f} GB/s) "
                       f"on the trace's durations. HIP events of the same (traced) run: "
                       f"{line['avg_launch_us']} us per launch.")
            if ref_path:
                for l in open(ref_path):
                    if l.startswith("{") and '"roofline"' in l:
                        ref = json.loads(l)["roofline"]
                        out.append(f"Unprofiled run with the same tile table: {ref['avg_launch_us']} us per launch "
                                   f"over {ref['launches']} launches (HIP events), {ref['achieved']} GB/s, "
                                   f"frac {ref['frac']}.")
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        a = agg[_short(r["Kernel_Name"])]
        a[0] += 1
        a[1] += dur(r)
    out.append("\n## whole run (including tile tuning), top 15 by total time\n")
    out.append("| calls | total ms | avg us | kernel |\n|---:|---:|---:|---|")
    for k, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:15]:
        out.append(f"| {n} | {t / 1000:.2f} | {t / n:.2f} | `{k}` |")
    return "\n".join(out) + "\n"


def act_step_positions(act, dur):
    """In-graph duration of each launch position of an act step (averaged over
    the steps of the replay, the first two and the last left out), grouped by
    kernel kind and convolution grid: which launches of the step take longest."""
    import collections
    steps, cur = [], []
    for r in act:
        if "prep_kernel<" in r["Kernel_Name"] and "core_prep" not in r["Kernel_Name"] and cur:
            steps.append(cur)
            cur = []
        cur.append(r)
    steps.append(cur)
    full = [s for s in steps[2:-1] if len(s) == len(steps[2])]
    if not full:
        return []
    n = len(full[0])
    avg = [sum(dur(s[i]) for s in full) / len(full) for i in range(n)]
    grp = collections.OrderedDict()
    for i in range(n):
        r = full[0][i]
        k = _short(r["Kernel_Name"])
        if "gemm_kernel" in k:
            k = f"{k.split(',')[0]}...> grid {r.get('Grid_Size_X', '?')}x{r.get('Grid_Size_Y', '?')}"
        g = grp.setdefault(k, [0, 0.0, []])
        g[0] += 1
        g[1] += avg[i]
        g[2].append(i)
    out = [f"\n## one act step by launch position ({n} launches, {len(full)} steps averaged): "
           f"kernel sum {sum(avg):.1f} us\n",
           "| launches per step | avg us | positions | kernel (GEMMs by grid: tiles x K splits) |",
           "|---:|---:|---|---|"]
    for k, (c, t, pos) in sorted(grp.items(), key=lambda kv: -kv[1][1] / kv[1][0]):
        out.append(f"| {c} | {t / c:.2f} | {','.join(map(str, pos[:8]))}{',...' if len(pos) > 8 else ''} | `{k}` |")
    return out


def summarize_counters(csv_path):
    """Per kernel class, summed counters of the dispatches after the landmark
    of a --pmc-probe run (the copy before it is the calibration): JSON."""
    import collections
    import csv
    rows = list(csv.DictReader(open(csv_path)))
    disp = collections.OrderedDict()
    for r in rows:
        d = disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"], "grid": r.get("Grid_Size", ""),
                                                     "c": collections.defaultdict(float)})
        d["c"][r["Counter_Name"]] += float(r["Counter_Value"])
    ids = sorted(disp)
    mark = [i for i in ids if disp[i]["name"].startswith("cast_bf16_kernel") and int(disp[i]["grid"] or 0) <= 256]
    copy = [i for i in ids if "copyBuffer" in disp[i]["name"]]
    cls = collections.defaultdict(lambda: {"dispatches": 0, "counters": collections.defaultdict(float)})
    start = mark[-1] if mark else -1
    for i in ids:
        if i <= start:
            continue
        name = disp[i]["name"]
        k = "conv forward GEMM" if "ConvFwdProb" in name else \
            "stem weight-gradient GEMM (channel-vector loads)" if "ConvWgradRTProb" in name else \
            "conv weight-gradient GEMM" if "ConvWgrad" in name \
            else "conv data-gradient GEMM" if "ConvDgrad" in name else "dense GEMM" if "DenseProb" in name \
            else _short(name)
        cls[k]["dispatches"] += 1
        for cn, v in disp[i]["c"].items():
            cls[k]["counters"][cn] += v
    calib = [{cn: v for cn, v in disp[i]["c"].items()} for i in ids if i < start and i in copy][:3]
    return {"copy_calibration": calib, "classes": {k: {"dispatches": v["dispatches"], **v["counters"]}
                                                    for k, v in cls.items()}}


# ---------------------------------------------------------------------- main
def main():
    if len(sys.argv) >= 3 and sys.argv[1] == "--summarize-trace":
        sys.stdout.write(summarize_trace(*sys.argv[2:5]))
        return
    if len(sys.argv) >= 3 and sys.argv[1] == "--summarize-counters":
        print(json.dumps(summarize_counters(sys.argv[2])))
        return
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
    from synth import rollout as R
    wl = WORKLOADS[a.workload]
    if a.pmc_probe:
        pmc_probe(wl, 0, a.pmc_probe, json.load(open(a.tiles_in)) if a.tiles_in else None)
        return
    seeds = list(range(a.seeds))
    progress(f"workload {a.workload}: selecting the dominant learner GEMM")
    sel = dominant_gemm(wl, 0)
    progress(f"timed runs, seeds {seeds[0]}..{seeds[-1]}")
    tiles = json.load(open(a.tiles_in)) if a.tiles_in else None
    res, w0 = run_seeds(wl, seeds, a.steps, a.warmup, wl.dtype, tiles)
    if a.tiles_out:
        with open(a.tiles_out, "w") as f:
            json.dump(w0.net.tile_table(), f)
    fps = [r["frames"] / (r["gpu_ms"] / 1e3) for r in res]
    value, ci = median_ci(fps)
    frames_step = res[0]["frames"] / a.steps
    ms_step = frames_step / value * 1e3
    out = {"metric": "PPO act+update frames/s", "value": round(value, 2), "unit": "frames/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16" if wl.dtype == "bf16" else "f32", "data": "synthetic",
           "config": {"workload": wl.name, "T": wl.T, "N": wl.N, "frame": f"{wl.net.in_ch}x{wl.net.in_hw}x{wl.net.in_hw}",
                      "encoder": encoder_label(wl.net),
                      "lstm": f"{wl.net.lstm_layers}x{wl.net.hidden}", "epochs": wl.ppo.epochs,
                      "minibatches": wl.ppo.minibatches, "frames_per_step": frames_step,
                      "parallelism": "single worker",
                      "gradient": "torch.autograd.Function, activations recomputed" if AUTOGRAD
                      else "ppo_loss_backward", "gemm_tiles": "autotuned in warm-up"},
           "seeds": len(seeds), "ci95": [round(c, 2) for c in ci],
           "health": {"adam_steps": sum(r["health"]["adam_steps"] for r in res),
                      "adam_skipped": sum(r["health"]["adam_skipped"] for r in res),
                      "loss_finite": all(r["health"]["loss_finite"] for r in res),
                      "recurrence_failed": any(r["health"]["recurrence_failed"] for r in res)},
           "per_seed": [round(x, 1) for x in fps],
           "wall_s": round(sum(r["wall_s"] for r in res), 3)}
    # roofline: the act step's convolution GEMMs (live, last timed replay of seed 0)
    roof = act_roofline(wl, res[0]["act"])
    env0, lens0 = stage_env(wl, 0, 0, torch.device("cuda", 0))
    learner = learner_gemm_live(w0, wl, env0, R.partitions(wl, 0), sel)
    learner["traffic"] = traffic_bytes(learner["kernel"], wl.name)
    net = w0.net
    w0.release()
    del w0, env0
    gc.collect()
    torch.cuda.empty_cache()
    progress("act / update split")
    act_ms, upd_ms, fr = act_update_split(wl, 0, net)
    del net
    out["act_ms"], out["update_ms"] = round(act_ms, 3), round(upd_ms, 3)
    out["act_frames_per_s"] = round((fr + wl.N) / (act_ms / 1e3), 1)
    out["update_frames_per_s"] = round(fr / (upd_ms / 1e3), 1)
    fpf = flops_per_frame(wl.net)
    upd_flops = 3 * fpf * fr * wl.ppo.epochs
    peak = PEAK_BF16_TFLOPS if wl.dtype == "bf16" else PEAK_FP32_TFLOPS
    # whole iteration: act forward of every frame (+ the bootstrap step) and E x (forward + backward)
    step_flops = fpf * ((1 + 3 * wl.ppo.epochs) * frames_step + wl.N)
    out["step_tflops"] = round(step_flops / (ms_step / 1e3) / 1e12, 3)
    out["step_mfma_frac"] = round(step_flops / (ms_step / 1e3) / 1e12 / peak, 5)
    out["update_tflops"] = round(upd_flops / (upd_ms / 1e3) / 1e12, 3)
    out["update_mfma_frac"] = round(upd_flops / (upd_ms / 1e3) / 1e12 / peak, 5)
    gc.collect()
    torch.cuda.empty_cache()
    if wl.dtype == "bf16" and not a.no_fp32:
        progress("float32 form, same seeds")
        r32, w32 = run_seeds(wl.with_(dtype="f32"), seeds, min(a.steps, 5), min(a.warmup, 2), "f32")
        w32.release()
        del w32
        f32 = [r["frames"] / (r["gpu_ms"] / 1e3) for r in r32]
        v32, ci32 = median_ci(f32)
        sp, cisp = median_ci(np.asarray(fps) / np.asarray(f32))
        out["fp32_value"] = round(v32, 2)
        out["fp32_ci95"] = [round(c, 2) for c in ci32]
        out["bf16_speedup_vs_fp32"] = round(sp, 3)
        out["bf16_speedup_ci95"] = [round(c, 3) for c in cisp]
        out["fp32_health"] = {"adam_skipped": sum(r["health"]["adam_skipped"] for r in r32),
                              "loss_finite": all(r["health"]["loss_finite"] for r in r32),
                              "recurrence_failed": any(r["health"]["recurrence_failed"] for r in r32)}
        gc.collect()
        torch.cuda.empty_cache()
    if wl.ragged:
        progress("unpacked per-env launches")
        ua, uu, ufr = unpacked_split(wl, 0)
        out["unpacked_act_frames_per_s"] = round((ufr + wl.N) / (ua / 1e3), 1)
        out["unpacked_update_frames_per_s"] = round(ufr / (uu / 1e3), 1)
        out["packed_speedup_act"] = round(out["act_frames_per_s"] / out["unpacked_act_frames_per_s"], 3)
        out["packed_speedup_update"] = round(out["update_frames_per_s"] / out["unpacked_update_frames_per_s"], 3)
        out["unpacked_gemm_tiles"] = "heuristic"
        gc.collect()
        torch.cuda.empty_cache()
    out["roofline"] = roof
    out["roofline_learner"] = learner
    if not a.no_cpu:
        progress("oracle CPU baseline and per-output errors")
        out["cpu_baseline"] = cpu_baseline(wl, 0)
    gc.collect()
    torch.cuda.synchronize()
    from paper_1911_00357_amd.api import live_nets
    out["library_handles_at_end"] = live_nets()   # 0: no graph, event or stream outlives the run
    print(json.dumps(out), flush=True)
    h, h32 = out["health"], out.get("fp32_health", {"adam_skipped": 0, "loss_finite": True, "recurrence_failed": False})
    if not h["loss_finite"] or h["recurrence_failed"] or (wl.dtype == "f32" and h["adam_skipped"]) or \
            not h32["loss_finite"] or h32["recurrence_failed"] or h32["adam_skipped"]:
        # a run whose updates were not all valid does not measure the method: say so and fail
        sys.stderr.write(f"bench: unhealthy run {h} (float32 form {h32})\n")
        sys.exit(3)


if __name__ == "__main__":
    main()
