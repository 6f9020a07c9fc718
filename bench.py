#!/usr/bin/env python3
"""Benchmark of the plain RT-CDF sort on one MI355X.

Workload (one "step"): sort each of the 15 arrays of the range sweep once:
n = 10^8 int32 keys, minVal = -1000, R in {2^7, 2^10, 2^13, 2^16, 2^18}, keys
uniform, normal (mean minVal + R/2, sd R/6, rounded, clamped) or all equal
(minVal + floor(R/3)).  Inputs are generated on the GPU from seeds and are
resident in HBM before timing starts; each sort writes its own output buffer.

Printed: one JSON line with the aggregate throughput (keys sorted per second
over the whole step), the per-case throughput and fraction of the 8 bytes/key
HBM roofline, a roofline entry for the dominant kernel measured with HIP events
inside the timed region, and the CPU oracle timed on this host (which also
checks every GPU output element by element).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published peak
N = 100_000_000
MIN_VAL = -1000
LOG_R = (7, 10, 13, 16, 18)
DISTS = ("uniform", "normal", "all_equal")
METRIC = "Gkeys/s + % of 8 B/key HBM roofline; batched & learned-tuned vs plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    p = os.path.join(ROOT, "paper_2609_00843_amd", "csrc", "rtcdf_kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(stage: str):
    """Counter-derived HBM bytes per launch for `stage`, if the counters were
    taken on the current kernel source (profiles/traffic.json), else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_sha():
        return None
    v = d.get("bytes_per_launch", {}).get(stage)
    return float(v) if v is not None else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cases", default="", help="comma list like 16:uniform,7:normal (default all)")
    ap.add_argument("--profile-only", action="store_true",
                    help="only run warmup + timed steps (for rocprofv3 runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              f"(the sort shards with one histogram all-reduce, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2609_00843_amd import inputs, rtcdf

    cases = [(lr, d) for lr in LOG_R for d in DISTS]
    if args.cases:
        want = {(int(a), b) for a, b in (c.split(":") for c in args.cases.split(","))}
        cases = [c for c in cases if c in want]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] generating {len(cases)} arrays of {N} keys on the GPU")
    ins, outs = [], []
    for i, (lr, d) in enumerate(cases):
        R = 1 << lr
        ins.append(inputs.make_device(d, N, MIN_VAL, MIN_VAL + R, inputs.case_seed(2, i), device=dev))
        outs.append(torch.empty(N, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def step():
        for (lr, _), a, b in zip(cases, ins, outs):
            rtcdf.sort(a, MIN_VAL, MIN_VAL + (1 << lr), keys_out=b, stream=stream)

    log(f"[bench] warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} steps")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    keys_step = N * len(cases)
    value = keys_step / (ms_step * 1e-3) / 1e9
    log(f"[bench] {ms_step:.4f} ms/step, {value:.1f} Gkeys/s (wall {wall / args.steps * 1e3:.4f} ms/step)")
    # Attainable-bandwidth reference: the library's plain copy of one input
    # array (N keys) into an output buffer, timed like a sort.
    cp0, cp1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        rtcdf.stream_copy(ins[0], outs[0], stream=stream)
    cp0.record(stream)
    for _ in range(args.steps):
        rtcdf.stream_copy(ins[0], outs[0], stream=stream)
    cp1.record(stream)
    torch.cuda.synchronize()
    copy_ms = cp0.elapsed_time(cp1) / args.steps
    copy_gbs = 8.0 * N / (copy_ms * 1e-3) / 1e9
    log(f"[bench] stream copy of {4 * N} bytes: {copy_ms:.4f} ms = {copy_gbs:.0f} GB/s (read + write)")
    if args.profile_only:
        print(json.dumps({"ms_per_step": ms_step, "value": value, "copy_ms": copy_ms}))
        return

    # Per-case times (same launches, one case at a time).
    per_case = []
    for (lr, d), a, b in zip(cases, ins, outs):
        R = 1 << lr
        for _ in range(3):
            rtcdf.sort(a, MIN_VAL, MIN_VAL + R, keys_out=b, stream=stream)
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(args.steps):
            rtcdf.sort(a, MIN_VAL, MIN_VAL + R, keys_out=b, stream=stream)
        c1.record(stream)
        torch.cuda.synchronize()
        ms = c0.elapsed_time(c1) / args.steps
        cfg = rtcdf.pick_config(N, MIN_VAL, MIN_VAL + R)
        per_case.append({"R": R, "dist": d, "ms": round(ms, 5),
                         "gkeys_per_s": round(N / (ms * 1e-3) / 1e9, 2),
                         "frac_8B_roofline": round(8.0 * N / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "config": list(cfg.as_tuple())})
        log(f"[bench] R=2^{lr:<2d} {d:9s} {ms:.4f} ms  {per_case[-1]['gkeys_per_s']:7.1f} Gkeys/s "
            f"{100 * per_case[-1]['frac_8B_roofline']:.1f}% of 8 B/key roofline")

    # Stage times with HIP events recorded by the library on the sort's stream.
    rtcdf.profile_collect()
    rtcdf.profile_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    st = rtcdf.profile_collect()
    rtcdf.profile_enable(False)
    nsorts = st["sorts"]
    stage_ms = {k: st[k] / max(nsorts, 1) for k in rtcdf.STAGES}
    dominant = "hist" if stage_ms["hist"] >= stage_ms["fill"] else "fill"
    algo_bytes = 4.0 * N        # hist reads every key once; fill writes every key once
    achieved = algo_bytes / (stage_ms[dominant] * 1e-3) / 1e9
    traffic = load_traffic(dominant)
    roofline = {"bound": "hbm", "kernel": "k_hist" if dominant == "hist" else "k_fill",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "algorithmic_bytes_per_launch": algo_bytes,
                "avg_launch_ms": round(stage_ms[dominant], 5)}
    other = "fill" if dominant == "hist" else "hist"
    roofline["other_kernel"] = {"kernel": "k_" + other, "avg_launch_ms": round(stage_ms[other], 5),
                                "achieved": round(algo_bytes / (stage_ms[other] * 1e-3) / 1e9, 1)}

    # CPU oracle on this host over the same arrays; doubles as a full parity check.
    cpu = None
    parity = "not checked"
    if not args.no_cpu_baseline:
        import oracle
        t_cpu, k_cpu, bad = 0.0, 0, []
        for (lr, d), a, b in zip(cases, ins, outs):
            R = 1 << lr
            A = a.cpu().numpy()
            t = time.perf_counter()
            B = oracle.sort(A, MIN_VAL, MIN_VAL + R)
            t_cpu += time.perf_counter() - t
            k_cpu += A.size
            if not np.array_equal(b.cpu().numpy(), B):
                bad.append(f"2^{lr}:{d}")
            del A, B
        parity = "bit-exact on all cases" if not bad else f"MISMATCH in {bad}"
        cpu = {"value": round(k_cpu / t_cpu / 1e9, 4), "unit": "Gkeys/s", "cores": 1,
               "kind": "oracle",
               "sample": f"all {len(cases)} arrays of the sweep at full size "
                         f"({k_cpu} keys), plain sequential counting sort, 1 thread, "
                         f"{os.cpu_count()} host cores visible"}
        log(f"[bench] oracle {cpu['value']} Gkeys/s on 1 core; parity: {parity}")

    tgt = [c for c in per_case if c["R"] <= (1 << 16)]
    rec = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "plain RT-CDF range sweep: n=1e8 int32 keys per array, minVal=-1000, "
                               "R in {2^7,2^10,2^13,2^16,2^18} x {uniform, normal sd R/6, all-equal}; "
                               "one step sorts all arrays",
                   "n": N, "arrays_per_step": len(cases), "keys_per_step": keys_step,
                   "parallelism": "single GPU"},
        "frac_8B_roofline_step": round(8.0 * keys_step / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "stream_copy_GBps": round(copy_gbs, 1),
        "min_frac_8B_roofline_R_le_2^16": round(min(c["frac_8B_roofline"] for c in tgt), 4) if tgt else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "stage_ms_per_sort": {k: round(v, 5) for k, v in stage_ms.items()},
        "cases": per_case,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
