"""Autotuning database, static default table and tuned table.

The database is append-only JSON lines, one row per measured array:
    {"key": ..., "n": ..., "minVal": ..., "R": ..., "dist": ..., "sd_div": ...,
     "features": [34 floats from the GPU sketch kernel],
     "times_ms": [one median per grid point from rtcdf_autotune, -1 for invalid ones]}
Rows are keyed by the array's seed, so an interrupted collection resumes where
it stopped.

The static default table follows the selection rule of Sec. 4.1 of the paper:
for every range class, the configuration with the smallest geometric mean of
t(config) / t_best over the arrays of that class.

Run ``python -m paper_2609_00843_amd.tune collect --set train --count 2000 --db PATH``
on a GPU, then ``python -m paper_2609_00843_amd.tune table --db PATH`` to write
csrc/rtcdf_default_table.h and the tuned table.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import inputs

PKG = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(PKG, "data")
TABLE_H = os.path.join(PKG, "csrc", "rtcdf_default_table.h")

GRID_T = [1024 << i for i in range(6)]
GRID_ITEMS = [4, 8, 16]
GRID_BPT = [1, 2, 4]
PLAIN_POINTS = 54
# option points (flags of rtcdf_config_t, on the static table's T / items /
# blocks): prefix-maximum output, 16-bit counters, 16-bit counters with wave
# aggregation of duplicates, wave aggregation, 4096-position output chunks,
# 16-bit counters with 4096-position chunks, 32-bit counters, 4-bit counters
GRID_OPTIONS = (0x01, 0x04, 0x14, 0x10, 0x20, 0x24, 0x08, 0x40)


def grid():
    """The grid points (T, items, blocks, flags) in library order and their
    validity: 54 plain points, then the option points as (0, 0, 0, flags)."""
    pts, valid = [], []
    for T in GRID_T:
        for it in GRID_ITEMS:
            for b in GRID_BPT:
                pts.append((T, it, b, 0))
                valid.append(T * 4 * b <= 163840)
    for f in GRID_OPTIONS:
        pts.append((0, 0, 0, f))
        valid.append(True)
    return pts, valid


SETS = {"train": 0, "test": 1, "heldout": 2}


def specs(which: str, count: int, seed: int = None):
    """Arrays like the single-array workloads: n log-uniform in [1e6, 1e9], R
    log-uniform in [2^7, 2^18] (rounded), minVal 0, keys uniform, normal with
    sd R/6, normal with sd R/64 or all equal; the held-out sets ("test", and
    "heldout", drawn from a seed no decision of the picker has seen) add
    Zipf(1.1)."""
    if seed is None:
        seed = inputs.case_seed(5, SETS[which])
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, 5])))
    dists = [("uniform", 6.0), ("normal", 6.0), ("normal", 64.0), ("all_equal", 6.0)]
    if which != "train":
        dists.append(("zipf", 6.0))
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(1e6), math.log(1e9)))))
        R = int(round(2.0 ** rng.uniform(7.0, 18.0)))
        d, sd = dists[int(rng.integers(0, len(dists)))]
        out.append({"key": f"{which}-{seed}-{i}", "n": n, "minVal": 0, "R": R, "dist": d, "sd_div": sd,
                    "seed": int(inputs.case_seed(6, i, seed))})
    return out


def load_db(path: str):
    rows = []
    if os.path.exists(path):
        with open(path) as f:
            for line in f:
                line = line.strip()
                if line:
                    rows.append(json.loads(line))
    return rows


def collect(db: str, which: str, count: int, warmup: int = 2, reps: int = 5, start: int = 0,
            stop: int = None, budget_s: float = None):
    """Measure every not-yet-measured array of the set; prints one line per array."""
    import torch
    from . import rtcdf
    done = {r["key"] for r in load_db(db)}
    todo = [s for s in specs(which, count)[start:stop] if s["key"] not in done]
    print(f"[tune] {len(done)} rows present, {len(todo)} to measure -> {db}", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(db)), exist_ok=True)
    dev = torch.device("cuda:0")
    t_start = time.time()
    with open(db, "a") as f:
        for k, s in enumerate(todo):
            if budget_s is not None and time.time() - t_start > budget_s:
                print(f"[tune] time budget reached after {k} arrays", flush=True)
                break
            a = inputs.make_device(s["dist"], s["n"], s["minVal"], s["minVal"] + s["R"], s["seed"],
                                   device=dev, sd_div=s["sd_div"])
            b = torch.empty_like(a)
            feats = rtcdf.sketch(a, s["minVal"], s["minVal"] + s["R"]).cpu().tolist()
            times, best = rtcdf.autotune(a, s["minVal"], s["minVal"] + s["R"], keys_out=b, warmup=warmup,
                                         reps=reps)
            row = dict(s)
            row["features"] = feats
            row["times_ms"] = times
            f.write(json.dumps(row) + "\n")
            f.flush()
            print(f"[tune] {k + 1}/{len(todo)} n={s['n']} R={s['R']} {s['dist']}/{s['sd_div']:g} "
                  f"best={best.as_tuple()} {min(t for t in times if t > 0):.4f} ms", flush=True)
            del a, b


def extend(db: str, out: str, warmup: int = 2, reps: int = 5, start: int = 0, stop: int = None):
    """Rows of `db` measured on a smaller grid get the times of the grid points
    added since (appended to times_ms, same protocol as rtcdf_autotune: the
    median of `reps` sorts, each between HIP events, after `warmup` untimed
    ones).  Rows [start, stop) are written to `out`, one per line as they are
    measured; rows already complete are copied."""
    import torch
    from . import rtcdf
    pts, valid = grid()
    rows = load_db(db)[start:stop]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    with open(out, "w") as f:
        for k, s in enumerate(rows):
            have = len(s["times_ms"])
            if have < len(pts):
                a = inputs.make_device(s["dist"], s["n"], s["minVal"], s["minVal"] + s["R"], s["seed"],
                                       device=dev, sd_div=s["sd_div"])
                b = torch.empty_like(a)
                for j in range(have, len(pts)):
                    if not valid[j]:
                        s["times_ms"].append(-1.0)
                        continue
                    cfg = rtcdf.make_config(*pts[j])
                    for _ in range(warmup):
                        rtcdf.sort(a, s["minVal"], s["minVal"] + s["R"], keys_out=b, config=cfg, stream=stream)
                    for e0, e1 in ev:
                        e0.record(stream)
                        rtcdf.sort(a, s["minVal"], s["minVal"] + s["R"], keys_out=b, config=cfg, stream=stream)
                        e1.record(stream)
                    torch.cuda.synchronize()
                    s["times_ms"].append(float(np.median([e0.elapsed_time(e1) for e0, e1 in ev])))
                del a, b
                print(f"[extend] {k + 1}/{len(rows)} n={s['n']} R={s['R']} {s['dist']}/{s['sd_div']:g} "
                      f"+{len(pts) - have} points: {s['times_ms'][have:]}", flush=True)
            f.write(json.dumps(s) + "\n")
            f.flush()


def range_class(R: int) -> int:
    return int(round(math.log2(R)))


def select_static(rows):
    """{range class: grid index} by the smallest geometric mean of t / t_best
    over the plain (T, items, blocks) points, the paper's grid."""
    _, valid = grid()
    by_class = {}
    for r in rows:
        by_class.setdefault(range_class(r["R"]), []).append(r)
    table = {}
    for c, rs in sorted(by_class.items()):
        scores = []
        for i in range(PLAIN_POINTS):
            if not valid[i]:
                scores.append(math.inf)
                continue
            logs = [math.log(r["times_ms"][i] /
                             min(t for t, v in zip(r["times_ms"][:PLAIN_POINTS], valid) if v))
                    for r in rs]
            scores.append(sum(logs) / len(logs))
        table[c] = int(np.argmin(scores))
    return table


# Ranges wider than the tuning rows (log2 R > 18.5): measured separately on
# MI355X over n in {10^7, 10^8}, R in {2^19 ... 2^24}, uniform and normal keys,
# where T = 8192 with 8 keys per thread was 0.80-0.98 x the time of the last
# tuned row's T = 1024 (the O(R) stages launch 8 x fewer tile workgroups).
WIDE_RANGE_CONFIG = (8192, 8, 1)


def write_default_table(table, path: str = TABLE_H, source: str = ""):
    pts, _ = grid()
    classes = sorted(table)
    lines = []
    for c in classes:
        # class c covers R up to the geometric midpoint towards class c + 1
        bound = f"{int(math.floor(2.0 ** (c + 0.5)))}u"
        T, it, b, _ = pts[table[c]]
        lines.append(f"    {{{bound}, {{{T}, {it}, {b}, 0}}}},   // log2 R ~ {c}")
    T, it, b = WIDE_RANGE_CONFIG
    lines.append(f"    {{1u << 28, {{{T}, {it}, {b}, 0}}}},   // wider than the tuning rows")
    body = "\n".join(lines)
    src = f"\n// Source: {source}" if source else ""
    text = f"""// rtcdf_default_table.h -- static default configuration per range class.
// Written by paper_2609_00843_amd/tune.py from measured tuning rows (the
// geometric mean of relative times per range, as in Sec. 4.1 of the paper);
// rows are ordered by max_range and the first row with R <= max_range applies.{src}
#pragma once

#include "../../include/rtcdf.h"

namespace rtcdf {{

struct DefaultRow {{
  uint32_t max_range;
  rtcdf_config_t cfg;
}};

static const DefaultRow kDefaultTable[] = {{
{body}
}};

}}  // namespace rtcdf
"""
    with open(path, "w") as f:
        f.write(text)


def write_tuned_table(rows, path: str):
    """One line per measured array: log2 n, log2 R and its fastest grid point
    (T items blocks flags; an option point as 0 0 0 flags)."""
    pts, valid = grid()
    with open(path, "w") as f:
        f.write("# log2n log2R T items blocks flags  (fastest measured grid point per array)\n")
        for r in rows:
            i = min((t, j) for j, t in enumerate(r["times_ms"]) if valid[j] and t > 0)[1]
            T, it, b, fl = pts[i]
            f.write(f"{math.log2(r['n']):.4f} {math.log2(r['R']):.4f} {T} {it} {b} {fl}\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--set", default="train", choices=sorted(SETS))
    c.add_argument("--count", type=int, default=2000)
    c.add_argument("--db", required=True)
    c.add_argument("--start", type=int, default=0)
    c.add_argument("--stop", type=int, default=None)
    c.add_argument("--budget-s", type=float, default=None)
    c.add_argument("--reps", type=int, default=5)
    e = sub.add_parser("extend")
    e.add_argument("--db", required=True)
    e.add_argument("--out", required=True)
    e.add_argument("--start", type=int, default=0)
    e.add_argument("--stop", type=int, default=None)
    e.add_argument("--reps", type=int, default=5)
    t = sub.add_parser("table")
    t.add_argument("--db", required=True)
    t.add_argument("--tuned-out", default=os.path.join(DATA, "tuned_table.txt"))
    args = ap.parse_args(argv)
    if args.cmd == "collect":
        collect(args.db, args.set, args.count, reps=args.reps, start=args.start, stop=args.stop,
                budget_s=args.budget_s)
    elif args.cmd == "extend":
        extend(args.db, args.out, reps=args.reps, start=args.start, stop=args.stop)
    else:
        rows = load_db(args.db)
        table = select_static(rows)
        write_default_table(table, source=f"{os.path.basename(args.db)}, {len(rows)} arrays")
        write_tuned_table(rows, args.tuned_out)
        print(json.dumps({str(k): grid()[0][v][:3] for k, v in table.items()}))


if __name__ == "__main__":
    sys.exit(main())
