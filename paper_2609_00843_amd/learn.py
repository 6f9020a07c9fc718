"""Training and evaluation of the learned configuration picker.

Inputs per array: the 34 sketch features (log2 n, log2 R, 32 bin fractions)
measured by the GPU sketch kernel.  Targets: for every valid grid
configuration, log(median runtime) minus the array's mean over its valid
configurations (only the ordering matters for the pick, and centring removes
the dependence of the scale on n).  The network is trained on the GPU by the
library's own kernels (rtcdf_mlp_train: full-batch Adam on the masked mean
squared error).

    python -m paper_2609_00843_amd.learn train --db TRAIN.jsonl --out MODEL.bin
    python -m paper_2609_00843_amd.learn evaluate --db TEST.jsonl --model MODEL.bin
    python -m paper_2609_00843_amd.learn heldout --model MODEL.bin --out EVAL.json

A checkpoint (.npz next to the model: weights, Adam moments, step, feature
normalisation, loss history) lets training resume.

The network's choice replaces the static table's only where it predicts at
least `margin` (natural-log units) less run time, and only for arrays whose
features lie within `zmax` standard deviations of the training mean in every
feature (zmax is twice the largest such distance among the fitting rows, the
factor fixed in advance): outside that the network is extrapolating and the
static table is kept.  The network is fitted on a seeded 80 % of the training
rows; on the other 20 % the margin with the best geometric-mean gain over the
static table is chosen (the larger one on ties).  The held-out test rows are
never used for fitting, for zmax or for the margin.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import struct
import sys

import numpy as np

from . import tune

NOUT = len(tune.grid()[0])          # one network output per grid point
SIZES = (34, 64, 64, NOUT)
NPARAMS = sum(SIZES[i + 1] * SIZES[i] + SIZES[i + 1] for i in range(3))
MODEL_VERSION = 4


def dataset(rows):
    _, valid = tune.grid()
    X = np.array([r["features"] for r in rows], dtype=np.float64)
    T = np.zeros((len(rows), NOUT))
    M = np.zeros((len(rows), NOUT))
    for i, r in enumerate(rows):
        t = np.array(r["times_ms"], dtype=np.float64)
        ok = np.array(valid) & (t > 0)
        lt = np.log(np.where(ok, t, 1.0))
        T[i] = np.where(ok, lt - lt[ok].mean(), 0.0)
        M[i] = ok
    return X, T, M


def normalisation(X):
    mu = X.mean(axis=0)
    sd = np.maximum(X.std(axis=0), 1e-3)
    return mu, sd


def init_params(seed: int):
    """He-initialised weights from a seeded generator (flat library layout)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(3):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / SIZES[i]), size=(SIZES[i + 1], SIZES[i])).ravel())
        parts.append(np.zeros(SIZES[i + 1]))
    return np.concatenate(parts).astype(np.float32)


MARGINS = tuple(round(0.005 * i, 3) for i in range(41))   # 0 .. 0.2


ZMAX_FACTOR = 2.0


def zmax_of(X, mu, sd) -> float:
    """Largest |normalised feature| over the rows of X."""
    return float(np.abs((np.asarray(X, dtype=np.float64) - mu) / sd).max())


def save_model(path: str, params, mu, sd, ranges, margin: float = 0.0, zmax: float = 0.0):
    """Model file version 4 (the grid with the 4-bit counter option point;
    version 1 had no margin and zmax fields, versions 1 and 2 the 54-point
    grid, version 3 the 61-point grid)."""
    _, valid = tune.grid()
    with open(path, "wb") as f:
        f.write(b"RTCDFMLP")
        f.write(struct.pack("<5I", MODEL_VERSION, 34, 64, NOUT, NPARAMS))
        f.write(struct.pack("<4f", *ranges))
        f.write(struct.pack("<2f", margin, zmax))
        f.write(np.asarray(mu, dtype=np.float32).tobytes())
        f.write(np.asarray(sd, dtype=np.float32).tobytes())
        f.write(np.asarray(params, dtype=np.float32).tobytes())
        f.write(bytes(1 if v else 0 for v in valid))


def train(rows, steps: int = 6000, lr: float = 3e-3, seed: int = 2609, chunk: int = 500,
          checkpoint: str = None, log=print):
    import torch
    from . import rtcdf
    X, T, M = dataset(rows)
    mu, sd = normalisation(X)
    Xn = (X - mu) / sd
    dev = torch.device("cuda:0")
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    Xd, Td, Md = f32(Xn), f32(T), f32(M)
    state = None
    if checkpoint and os.path.exists(checkpoint):
        state = np.load(checkpoint)
    P = f32(state["params"] if state is not None else init_params(seed))
    m = f32(state["m"]) if state is not None else torch.zeros_like(P)
    v = f32(state["v"]) if state is not None else torch.zeros_like(P)
    t = int(state["t"]) if state is not None else 0
    hist = list(state["loss"]) if state is not None else []
    ws = rtcdf.mlp_workspace(X.shape[0], dev)
    while t < steps:
        k = min(chunk, steps - t)
        lh = torch.empty(k, dtype=torch.float32, device=dev)
        rtcdf.mlp_train(P, m, v, t, Xd, Td, Md, k, lr, ws=ws, loss_history=lh)
        t += k
        hist.extend(lh.cpu().tolist())
        log(f"[learn] step {t}/{steps} loss {hist[-1]:.5f}")
        if checkpoint:
            np.savez(checkpoint, params=P.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(), t=t,
                     mu=mu, sd=sd, loss=np.array(hist))
    ranges = (float(X[:, 0].min()), float(X[:, 0].max()), float(X[:, 1].min()), float(X[:, 1].max()))
    return P.cpu().numpy(), mu, sd, ranges, hist


def predict(params, mu, sd, X):
    """Network outputs for feature rows X, computed by the library's kernel."""
    import torch
    from . import rtcdf
    dev = torch.device("cuda:0")
    Xn = torch.from_numpy(((X - mu) / sd).astype(np.float32)).to(dev)
    P = torch.from_numpy(np.asarray(params, dtype=np.float32)).to(dev)
    return rtcdf.mlp_forward(P, Xn).cpu().numpy()


def load_model_file(path: str):
    """(params, mean, sd, ranges, margin, zmax) of a model file of version 1,
    2 or 3 (its parameter count is read from the header)."""
    with open(path, "rb") as f:
        raw = f.read()
    assert raw[:8] == b"RTCDFMLP"
    version, _, _, _, nparams = struct.unpack("<5I", raw[8:28])
    assert version in (1, 2, 3, 4)
    o = 8 + 20
    ranges = struct.unpack("<4f", raw[o:o + 16])
    o += 16
    margin = zmax = 0.0
    if version >= 2:
        margin, zmax = struct.unpack("<2f", raw[o:o + 8])
        o += 8
    mu = np.frombuffer(raw, dtype=np.float32, count=34, offset=o).astype(np.float64)
    o += 136
    sd = np.frombuffer(raw, dtype=np.float32, count=34, offset=o).astype(np.float64)
    o += 136
    params = np.frombuffer(raw, dtype=np.float32, count=nparams, offset=o).copy()
    return params, mu, sd, ranges, margin, zmax


def static_indices(rows):
    """Grid index of the static choice for every row (the library's DEFAULT
    pick: the static table and the output-method rule; host logic only)."""
    from . import rtcdf
    old = rtcdf.get_config_mode()
    rtcdf.set_config_mode(rtcdf.CONFIG_DEFAULT)
    try:
        out = []
        for r in rows:
            rtcdf.pick_config(r["n"], r["minVal"], r["minVal"] + r["R"])
            out.append(rtcdf.last_pick()[0])
        return out
    finally:
        rtcdf.set_config_mode(old)


def decide(y, ok, static: int, margin: float, trusted: bool = True) -> int:
    """The network's masked argmin where the array's features are trusted and
    it predicts at least `margin` less than for the static choice, else the
    static choice."""
    if not trusted:
        return static
    pick = min((y[j], j) for j in range(len(y)) if ok[j])[1]
    if ok[static] and y[static] - y[pick] < margin:
        return static
    return pick


def margin_gains(Y, rows, statics, trusted=None):
    """Geometric-mean gain over the static choice, on the rows' measured
    times, of every margin in MARGINS."""
    _, valid = tune.grid()
    trusted = trusted if trusted is not None else [True] * len(rows)
    out = []
    for mg in MARGINS:
        logs = []
        for r, y, si, tr in zip(rows, Y, statics, trusted):
            t = np.array(r["times_ms"])
            ok = np.array(valid) & (t > 0)
            logs.append(math.log(t[si] / t[decide(y, ok, si, mg, tr)]))
        out.append(math.exp(sum(logs) / len(logs)))
    return out


def choose_margin(Y, rows, statics, trusted=None):
    """The margin (from MARGINS) with the best geometric-mean gain over the
    static choice on the rows' measured times; the larger margin on ties."""
    gains = margin_gains(Y, rows, statics, trusted)
    best = (None, -1.0)
    for mg, g in zip(MARGINS, gains):
        if g >= best[1]:
            best = (mg, g)
    return best


def evaluate(rows, model_path: str):
    """Regret of the learned pick against the exhaustive optimum of the same
    (independent) timing run, and its gain over the static default table,
    with the model's margin and feature gate applied."""
    params, mu, sd, _, margin, zmax = load_model_file(model_path)
    pts, valid = tune.grid()
    X = np.array([r["features"] for r in rows], dtype=np.float64)
    Y = predict(params, mu, sd, X)
    statics = static_indices(rows)
    trusted = [zmax <= 0 or zmax_of(x[None, :], mu, sd) <= zmax for x in X]
    regrets, gains, per = [], [], []
    for r, y, static, tr in zip(rows, Y, statics, trusted):
        t = np.array(r["times_ms"])
        ok = np.array(valid) & (t > 0)
        pick = decide(y, ok, static, margin, tr)
        best = float(t[ok].min())
        regrets.append(t[pick] / best - 1.0)
        gains.append(t[static] / t[pick])
        per.append({"key": r["key"], "dist": r["dist"], "n": r["n"], "R": r["R"], "pick": pts[pick],
                    "static": pts[static], "t_pick": float(t[pick]), "t_static": float(t[static]),
                    "t_best": best, "trusted": bool(tr)})
    reg = np.array(regrets)
    res = {"arrays": len(rows), "margin": margin, "zmax": zmax,
           "within_zmax": float(np.mean(trusted)),
           "learned_choice_used": float(np.mean([p["pick"] != p["static"] for p in per])),
           "regret_mean": float(reg.mean()), "regret_median": float(np.median(reg)),
           "regret_p95": float(np.percentile(reg, 95)), "regret_max": float(reg.max()),
           "gain_geomean_vs_static": float(np.exp(np.mean(np.log(gains)))),
           "static_regret_mean": float(np.mean([p["t_static"] / p["t_best"] - 1 for p in per]))}
    by_dist = {}
    for p, g, rg in zip(per, gains, regrets):
        by_dist.setdefault(p["dist"], []).append((g, rg))
    res["by_dist"] = {d: {"gain_geomean": float(np.exp(np.mean(np.log([g for g, _ in v])))),
                          "regret_mean": float(np.mean([rg for _, rg in v])), "arrays": len(v)}
                      for d, v in by_dist.items()}
    return res, per


def time_config(torch, rtcdf, a, b, lo, hi, cfg, warmup=10, reps=30, runs=3):
    """Median over `runs` runs of the median of `reps` sorts, each bracketed by
    HIP events on the stream, after `warmup` untimed sorts (the paper's
    protocol: the median of 3 run-medians of 30 after 10 warm-ups)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        rtcdf.sort(a, lo, hi, keys_out=b, config=cfg, stream=stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    meds = []
    for _ in range(runs):
        for e0, e1 in ev:
            e0.record(stream)
            rtcdf.sort(a, lo, hi, keys_out=b, config=cfg, stream=stream)
            e1.record(stream)
        torch.cuda.synchronize()
        meds.append(float(np.median([e0.elapsed_time(e1) for e0, e1 in ev])))
    return float(np.median(meds))


PICK_NAMES = {0: "static", 1: "network", 2: "network_kept_static", 3: "autotuned", 4: "cached", 5: "pending"}


def evaluate_retimed(specs, model_path: str, warmup: int = 10, reps: int = 30, runs: int = 3,
                     tune_reps: int = 5, log=print):
    """Held-out evaluation with every time measured in this run, on the GPU.
    Per array (generated on the device from its spec):
      1. exhaustive autotuning of the whole grid (the reference that regret is measured against);
      2. the library's LEARNED decision from a cold decision cache (its pick
         time measured, including any exhaustive fallback), and the time of
         the same call once the decision is cached;
      3. the static choice (DEFAULT mode), the learned choice and the
         exhaustive best re-timed by time_config (median of run-medians).
    Gain = t(static) / t(learned) (steady state: the decision made once); the
    gains with one cold pick per K sorts are reported beside it."""
    import time
    import torch
    from . import inputs, rtcdf
    pts, valid = tune.grid()
    rtcdf.load_model(model_path)
    old = rtcdf.get_config_mode()
    per = []
    try:
        for k, s in enumerate(specs):
            n, lo = s["n"], s["minVal"]
            hi = lo + s["R"]
            a = inputs.make_device(s["dist"], n, lo, hi, s["seed"], sd_div=s["sd_div"])
            b = torch.empty_like(a)
            torch.cuda.synchronize()
            rtcdf.set_config_mode(rtcdf.CONFIG_DEFAULT)
            cfg_s = rtcdf.pick_config(n, lo, hi)
            i_s = rtcdf.last_pick()[0]
            times, _ = rtcdf.autotune(a, lo, hi, keys_out=b, warmup=2, reps=tune_reps)
            i_b = min((t, j) for j, t in enumerate(times) if valid[j] and t > 0)[1]
            rtcdf.set_config_mode(rtcdf.CONFIG_LEARNED)
            rtcdf.clear_pick_cache()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cfg_l = rtcdf.pick_config(n, lo, hi, keys_in=a)
            pick_ms = (time.perf_counter() - t0) * 1e3
            i_l, src = rtcdf.last_pick()
            t0 = time.perf_counter()
            rtcdf.pick_config(n, lo, hi, keys_in=a)
            cached_ms = (time.perf_counter() - t0) * 1e3
            rtcdf.set_config_mode(rtcdf.CONFIG_DEFAULT)
            cfg_b = rtcdf.make_config(*pts[i_b])
            memo = {}

            def t_of(cfg):
                key = cfg.as_tuple()
                if key not in memo:
                    memo[key] = time_config(torch, rtcdf, a, b, lo, hi, cfg, warmup, reps, runs)
                return memo[key]

            ts, tl, tb = t_of(cfg_s), t_of(cfg_l), t_of(cfg_b)
            row = {"key": s["key"], "dist": s["dist"] if s["dist"] != "normal" else f"normal/{s['sd_div']:g}",
                   "n": n, "R": s["R"], "static": i_s, "learned": i_l, "best": i_b,
                   "source": PICK_NAMES.get(src, src), "t_static": ts, "t_learned": tl, "t_best": tb,
                   "t_best_autotune": float(times[i_b]), "pick_ms": pick_ms, "cached_pick_ms": cached_ms,
                   "features": rtcdf.sketch(a, lo, hi).cpu().tolist()}
            per.append(row)
            log(f"[heldout] {k + 1}/{len(specs)} n={n} R={s['R']} {row['dist']} {row['source']}: static "
                f"{ts:.4f} learned {tl:.4f} best {tb:.4f} ms (pick {pick_ms:.3f} ms)")
            del a, b
    finally:
        rtcdf.set_config_mode(old)
    return summarise_retimed(per), per


def summarise_retimed(per):
    """Gain, regret and pick-cost summary of evaluate_retimed's rows, overall,
    per distribution and per decision source."""
    def block(rows):
        if not rows:
            return None
        g = np.array([r["t_static"] / r["t_learned"] for r in rows])
        reg = np.array([r["t_learned"] / r["t_best"] - 1.0 for r in rows])
        sreg = np.array([r["t_static"] / r["t_best"] - 1.0 for r in rows])
        out = {"arrays": len(rows), "gain_geomean": float(np.exp(np.log(g).mean())),
               "regret_mean": float(reg.mean()), "regret_median": float(np.median(reg)),
               "regret_p95": float(np.percentile(reg, 95)), "regret_max": float(reg.max()),
               "static_regret_mean": float(sreg.mean()),
               "learned_differs": float(np.mean([r["learned"] != r["static"] for r in rows]))}
        for K in (1, 10, 100):
            gk = [r["t_static"] / (r["t_learned"] + r["pick_ms"] / K) for r in rows]
            out[f"gain_geomean_one_pick_per_{K}_sorts"] = float(np.exp(np.mean(np.log(gk))))
        out["pick_ms_median"] = float(np.median([r["pick_ms"] for r in rows]))
        out["cached_pick_ms_median"] = float(np.median([r["cached_pick_ms"] for r in rows]))
        return out
    res = block(per)
    res["by_dist"] = {d: block([r for r in per if r["dist"] == d]) for d in sorted({r["dist"] for r in per})}
    res["by_source"] = {s: block([r for r in per if r["source"] == s])
                        for s in sorted({r["source"] for r in per})}
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--db", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--steps", type=int, default=6000)
    t.add_argument("--lr", type=float, default=3e-3)
    t.add_argument("--seed", type=int, default=2609)
    e = sub.add_parser("evaluate")
    e.add_argument("--db", required=True)
    e.add_argument("--model", required=True)
    e.add_argument("--out", default=None)
    h = sub.add_parser("heldout", help="re-timed evaluation on a held-out set generated on the GPU")
    h.add_argument("--model", required=True)
    h.add_argument("--set", default="heldout")
    h.add_argument("--count", type=int, default=500)
    h.add_argument("--start", type=int, default=0)
    h.add_argument("--stop", type=int, default=None)
    h.add_argument("--out", required=True)
    m = sub.add_parser("merge", help="one summary over several heldout result files")
    m.add_argument("parts", nargs="+")
    m.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "merge":
        per = []
        for path in args.parts:
            with open(path) as f:
                per.extend(json.load(f)["arrays"])
        res = summarise_retimed(per)
        with open(args.out, "w") as f:
            json.dump({"summary": res, "arrays": per}, f)
        print(json.dumps({k: v for k, v in res.items() if k not in ("by_dist", "by_source")}))
        return 0
    if args.cmd == "heldout":
        specs = tune.specs(args.set, args.count)[args.start:args.stop]
        res, per = evaluate_retimed(specs, args.model, log=lambda *a: print(*a, flush=True))
        with open(args.out, "w") as f:
            json.dump({"summary": res, "arrays": per}, f)
        print(json.dumps({k: v for k, v in res.items() if k not in ("by_dist", "by_source")}))
        return 0
    if args.cmd == "train":
        rows = tune.load_db(args.db)
        order = np.random.default_rng(args.seed).permutation(len(rows))
        n_val = len(rows) // 5
        val = [rows[i] for i in order[:n_val]]
        fit = [rows[i] for i in order[n_val:]]
        params, mu, sd, ranges, hist = train(fit, steps=args.steps, lr=args.lr, seed=args.seed,
                                             checkpoint=os.path.splitext(args.out)[0] + "_ckpt.npz")
        zmax = ZMAX_FACTOR * zmax_of([r["features"] for r in fit], mu, sd)
        Xv = np.array([r["features"] for r in val], dtype=np.float64)
        trusted = [zmax_of(x[None, :], mu, sd) <= zmax for x in Xv]
        margin, gain = choose_margin(predict(params, mu, sd, Xv), val, static_indices(val), trusted)
        save_model(args.out, params, mu, sd, ranges, margin, zmax)
        print(json.dumps({"rows_fit": len(fit), "rows_validation": len(val), "final_loss": hist[-1],
                          "first_loss": hist[0], "margin": margin, "zmax": zmax,
                          "validation_gain": gain, "model": args.out}))
    else:
        res, per = evaluate(tune.load_db(args.db), args.model)
        if args.out:
            with open(args.out, "w") as f:
                json.dump({"summary": res, "arrays": per}, f)
        print(json.dumps(res))


if __name__ == "__main__":
    sys.exit(main())
