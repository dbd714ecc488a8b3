"""Shared helpers of the GPU parity tests: seeded rollout records in the
library's layout, the matching oracle minibatch, and per-tensor errors."""
import numpy as np
import torch

from synth import rollout as R
from synth.layout import tensor_list

DEV = "cuda"


def rel_err(x, ref, floor=1e-30):
    x, ref = np.asarray(x, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), floor))


def per_tensor_errors(net, g, g_ref):
    """{tensor name: relative L2 error} over the flat layout."""
    out = {}
    for t in tensor_list(net):
        n = int(np.prod(t.shape))
        sl = slice(t.offset, t.offset + n)
        out[t.name] = rel_err(g[sl], g_ref[sl], floor=1e-12)
    return out


def random_record(net, T, N, seed, lengths=None, bf16=False, logp_spread=0.3):
    """A synthetic rollout record [T+1][N] (act-step arrays) / [T][N]
    (transition arrays).  Old log-probs are random so both clip branches of
    the surrogate occur."""
    g = np.random.default_rng(seed)
    obs = g.random((T + 1, N, net.in_ch, net.in_hw, net.in_hw), dtype=np.float32)
    if bf16:
        obs = R.round_bf16(obs)
    act = g.integers(0, net.num_actions, (T + 2, N)).astype(np.int32)
    return {
        "obs": obs,
        "goal": g.standard_normal((T + 1, N, 2)).astype(np.float32),
        "mask": (g.random((T + 1, N)) > 0.15).astype(np.float32),
        "act_rec": act,
        "logp": (np.log(0.25) + logp_spread * g.standard_normal((T + 1, N))).astype(np.float32),
        "adv": g.standard_normal((T, N)).astype(np.float32),
        "ret": g.standard_normal((T, N)).astype(np.float32),
        "h0": (0.5 * g.standard_normal((net.lstm_layers, N, net.hidden))).astype(np.float32),
        "c0": (0.5 * g.standard_normal((net.lstm_layers, N, net.hidden))).astype(np.float32),
        "lengths": np.full(N, T, np.int32) if lengths is None else np.asarray(lengths, np.int32),
    }


def to_device(rec, bf16=False):
    t = lambda a, dt=None: torch.as_tensor(np.ascontiguousarray(a)).to(DEV) if dt is None else \
        torch.as_tensor(np.ascontiguousarray(a)).to(DEV).to(dt)
    act = t(rec["act_rec"])
    return {
        "obs": t(rec["obs"], torch.bfloat16 if bf16 else torch.float32),
        "goal": t(rec["goal"]), "mask": t(rec["mask"]),
        "prev_action": act[:-1], "action": act[1:], "logp": t(rec["logp"]),
        "adv": t(rec["adv"]), "ret": t(rec["ret"]), "h0": t(rec["h0"]), "c0": t(rec["c0"]),
    }


def oracle_minibatch(rec, envs):
    """The oracle's minibatch dict for env set `envs` (time-major [T_B, B])."""
    envs = np.asarray(envs)
    lens = rec["lengths"][envs]
    TB = int(lens.max())
    a = rec["act_rec"]
    return {
        "envs": envs, "lens": lens,
        "obs": rec["obs"][:TB][:, envs].astype(np.float64),
        "goal": rec["goal"][:TB][:, envs].astype(np.float64),
        "prev_action": a[:TB][:, envs], "mask": rec["mask"][:TB][:, envs].astype(np.float64),
        "action": a[1:TB + 1][:, envs], "logp_old": rec["logp"][:TB][:, envs].astype(np.float64),
        "adv": rec["adv"][:TB][:, envs].astype(np.float64),
        "ret": rec["ret"][:TB][:, envs].astype(np.float64),
        "h0": rec["h0"][:, envs].astype(np.float64), "c0": rec["c0"][:, envs].astype(np.float64),
    }


# ------------------------------------------------------------ comparisons
def errs(x, ref):
    """(relative L2, max |x - ref| / max |ref|) of one output."""
    x, ref = np.asarray(x, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    if ref.size == 0:
        return 0.0, 0.0
    d = np.abs(x - ref)
    return (float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-30)),
            float(d.max() / max(np.abs(ref).max(), 1e-30)))


def assert_close(name, x, ref, tol):
    """Relative L2 and element-wise (max abs error over max abs value)
    errors both within tol; returns them."""
    l2, mx = errs(x, ref)
    assert l2 < tol and mx < tol, f"{name}: relative L2 {l2:.2e}, element-wise {mx:.2e} (tol {tol:.0e})"
    return l2, mx


def tensor_errors(net, g, g_ref):
    """{tensor name: (relative L2, element-wise)} over the flat layout."""
    out = {}
    for t in tensor_list(net):
        n = int(np.prod(t.shape))
        sl = slice(t.offset, t.offset + n)
        out[t.name] = errs(g[sl], g_ref[sl])
    return out


def _windows3s2(x):
    """[F,C,H,W] -> [F,C,Ho,Wo,9] windows of the 3x3 / stride 2 / pad 1 max pool
    (padding -inf), window index kh*3+kw."""
    F_, C, H, W = x.shape
    Ho, Wo = (H - 1) // 2 + 1, (W - 1) // 2 + 1
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)), constant_values=-np.inf)
    v = np.lib.stride_tricks.sliding_window_view(xp, (3, 3), axis=(2, 3))
    return v[:, :, 0:2 * (Ho - 1) + 1:2, 0:2 * (Wo - 1) + 1:2].reshape(F_, C, Ho, Wo, 9)


def validate_decisions(dec, rec, lens, tol, qtol=None):
    """Every imposed decision that differs from the one the oracle would take
    at the same point must sit at a near-kink.  rec: the oracle's record of a
    run with `dec` imposed (pre-activations under those decisions).  A ReLU
    whose imposed on/off state disagrees with the sign of its pre-activation
    y needs |y| <= tol * rms(y of its tensor); an imposed max-pool winner
    below its window's maximum needs the gap <= tol * rms(pool input); an
    imposed bfloat16 operand code ('q:' keys) must be the rounding of some
    value within qtol * rms(x) of the oracle's own value x (a code other than
    round(x) only where x sits that close to a rounding midpoint).
    Returns {key: (units, flips)}; raises with the worst offender otherwise."""
    from oracle.nn import round_bf16
    out = {}
    bad = []
    for key, m in dec.items():
        if key.startswith("q:"):
            x, c = rec[key], np.asarray(m, np.float64)
            if key.startswith("q:fc") or key.startswith("q:lstm"):     # time-major, valid frames
                valid = np.arange(x.shape[0])[:, None] < np.asarray(lens)[None, :]
                x, c = x[valid], c[valid]
            tau = qtol * np.sqrt(np.mean(x * x))
            lo, hi = round_bf16(x - tau), round_bf16(x + tau)
            flips = int(np.count_nonzero(c != round_bf16(x)))
            out[key] = (x.size, flips)
            outside = (c < lo) | (c > hi)
            if outside.any():
                i = np.flatnonzero(outside.ravel())[0]
                bad.append((key, float(x.ravel()[i]), float(c.ravel()[i]), int(outside.sum())))
            continue
        if key == "maxpool":
            x = rec["maxpool"]
            win = _windows3s2(x)
            k = np.asarray(m, np.int64)
            assert k.min() >= 0 and k.max() <= 8, "winner index outside the window"
            chosen = np.take_along_axis(win, k[..., None], axis=4)[..., 0]
            assert np.isfinite(chosen).all(), "a winner points at padding"
            gap = win.max(axis=4) - chosen
            scale = np.sqrt(np.mean(x * x))
            flips = int(np.count_nonzero(gap > 0))
            worst = float(gap.max()) / scale
            out[key] = (gap.size, flips)
        else:
            y = rec[key]
            m = np.asarray(m, bool)
            if key == "vis":
                valid = np.arange(y.shape[0])[:, None] < np.asarray(lens)[None, :]
                y, m = y[valid], m[valid]
            scale = np.sqrt(np.mean(y * y))
            diff = (y > 0) != m
            flips = int(np.count_nonzero(diff))
            worst = float(np.abs(y[diff]).max()) / scale if flips else 0.0
            out[key] = (y.size, flips)
        if worst > tol:
            bad.append((key, worst, flips))
    assert not bad, f"imposed decisions far from a kink (key, margin / rms, flips): {bad} (tol {tol})"
    return out


def flip_summary(fl):
    units = sum(u for u, _ in fl.values())
    flips = sum(f for _, f in fl.values())
    top = sorted(fl.items(), key=lambda kv: -kv[1][1])[:3]
    return (f"{flips} of {units} decisions flipped ({flips / max(units, 1):.1e})" +
            ("; most in " + ", ".join(f"{k}={f}" for k, (_, f) in top if f) if flips else ""))
