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
PICK_NAMES = {0: "static", 1: "network", 2: "network_kept_static", 3: "autotuned", 4: "cached", 5: "pending"}
WIDE_LOG_R = (20, 22, 24)   # beyond the paper's ranges: the partition by pass
DISTS = ("uniform", "normal", "all_equal")
METRIC = "Gkeys/s + % of 8 B/key HBM roofline; batched & learned-tuned vs plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    """Hash of the sources the plain-sort kernels are compiled from."""
    h = hashlib.sha256()
    for f in ("rtcdf_kernels.hip", "rtcdf_device.h", "rtcdf_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2609_00843_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """Counter-derived HBM bytes per launch of `kernel` over the sweep, if the
    counters were taken on the current kernel source (profiles/traffic.json),
    else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_sha():
        return None
    v = d.get("bytes_per_launch", {}).get(kernel)
    return float(v) if v is not None else None


def bench_batched(torch, rtcdf, inputs, steps, check):
    """The 4096-array batch workload: one HIP-graph launch of the batched sort
    against the same arrays sorted by 4096 plain calls (eagerly, and captured in
    one graph through the caller-workspace entry point)."""
    import numpy as np
    segs = inputs.batched_segments(4096)
    total = sum(s["n"] for s in segs)
    dev = torch.device("cuda:0")
    din = torch.empty(total, dtype=torch.int32, device=dev)
    dout = torch.empty(total, dtype=torch.int32, device=dev)
    pairs, o = [], 0
    for s in segs:
        n = s["n"]
        din[o:o + n] = inputs.make_device(s["dist"], n, s["minVal"], s["maxVal"], s["seed"], device=dev)
        pairs.append((din[o:o + n], dout[o:o + n], s["minVal"], s["maxVal"]))
        o += n
    torch.cuda.synchronize()
    # Everything is timed on torch's current stream, where graph replays run.
    stream = torch.cuda.current_stream()
    d, bounds, k = rtcdf.make_segments(pairs)
    ws = torch.empty(rtcdf.batched_workspace_bytes(k, bounds), dtype=torch.uint8, device=dev)
    rtcdf.sort_batched(d, k, bounds, ws, stream=stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rtcdf.sort_batched(d, k, bounds, ws, stream=torch.cuda.current_stream())

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    dout.fill_(0)
    t_batched = timed(g.replay, steps)
    parity = "not checked"
    # Part of the CPU (oracle) leg: skipped together with it by --no-cpu-baseline.
    if check:
        import oracle
        outs = dout.cpu().numpy()
        ins = din.cpu().numpy()
        bad, o = 0, 0
        for s in segs:
            n = s["n"]
            if not np.array_equal(outs[o:o + n], oracle.sort(ins[o:o + n], s["minVal"], s["maxVal"])):
                bad += 1
            o += n
        parity = "bit-exact on all 4096 arrays" if bad == 0 else f"MISMATCH in {bad} arrays"
        del outs, ins

    def plain_loop():
        for a, b, lo, hi in pairs:
            rtcdf.sort(a, lo, hi, keys_out=b, stream=stream)

    t_plain = timed(plain_loop, max(1, steps // 5))
    # the same plain sorts in one captured graph, sharing one caller workspace
    wsz = max(rtcdf.workspace_bytes(a.numel(), lo, hi, keys_out=b) for a, b, lo, hi in pairs)
    pws = torch.empty(wsz, dtype=torch.uint8, device=dev)
    for a, b, lo, hi in pairs:
        rtcdf.sort_ws(a, b, lo, hi, pws, stream=stream)
    torch.cuda.synchronize()
    pg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(pg):
        cs = torch.cuda.current_stream()
        for a, b, lo, hi in pairs:
            rtcdf.sort_ws(a, b, lo, hi, pws, stream=cs)
    t_plain_graph = timed(pg.replay, max(1, steps // 5))
    gk = lambda ms: round(total / (ms * 1e-3) / 1e9, 2)
    return {"workload": "4096 int32 arrays: n log-uniform in [1e3,1e6], minVal uniform in [-1e6,1e6], "
                        "R log-uniform in [2^4,2^16], uniform / normal sd R/6 / all-equal",
            "keys": total, "ms_batched_graph": round(t_batched, 4), "gkeys_per_s": gk(t_batched),
            "frac_8B_roofline": round(8.0 * total / (t_batched * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "ms_plain_calls": round(t_plain, 4), "gkeys_per_s_plain_calls": gk(t_plain),
            "ms_plain_graph": round(t_plain_graph, 4), "gkeys_per_s_plain_graph": gk(t_plain_graph),
            "speedup_vs_plain_calls": round(t_plain / t_batched, 2),
            "speedup_vs_plain_graph": round(t_plain_graph / t_batched, 2), "parity": parity}


def profile_batched(torch, rtcdf, inputs, steps, warmup):
    """Profiling mode: the 4096-array batched workload, `warmup` then `steps`
    graph replays (one launch of the ordering kernel and one of k_batched
    each), then the copy reference of the counter calibration."""
    segs = inputs.batched_segments(4096)
    total = sum(s["n"] for s in segs)
    dev = torch.device("cuda:0")
    din = torch.empty(total, dtype=torch.int32, device=dev)
    dout = torch.empty(total, dtype=torch.int32, device=dev)
    pairs, o = [], 0
    for s in segs:
        n = s["n"]
        din[o:o + n] = inputs.make_device(s["dist"], n, s["minVal"], s["maxVal"], s["seed"], device=dev)
        pairs.append((din[o:o + n], dout[o:o + n], s["minVal"], s["maxVal"]))
        o += n
    d, bounds, k = rtcdf.make_segments(pairs)
    ws = torch.empty(rtcdf.batched_workspace_bytes(k, bounds), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    rtcdf.sort_batched(d, k, bounds, ws, stream=stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rtcdf.sort_batched(d, k, bounds, ws, stream=torch.cuda.current_stream())
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    log(f"[bench] batched: {ms:.4f} ms per replay, {total / (ms * 1e-3) / 1e9:.1f} Gkeys/s")
    src = torch.empty(N, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(steps):
        rtcdf.stream_copy(src, dst, stream=stream)
    torch.cuda.synchronize()
    print(json.dumps({"ms_per_step": ms, "keys_per_step": total}))


def timed_sorts(torch, rtcdf, a, b, lo, hi, reps, stream, config=None):
    for _ in range(3):
        rtcdf.sort(a, lo, hi, keys_out=b, stream=stream, config=config)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        rtcdf.sort(a, lo, hi, keys_out=b, stream=stream, config=config)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_small(torch, rtcdf, inputs, steps):
    """n = 10^6 uniform keys in [0, 128): launch-latency bound; warm timing
    (input and output stay in the last-level cache between sorts)."""
    dev = torch.device("cuda:0")
    n, R = 1_000_000, 128
    a = inputs.make_device("uniform", n, 0, R, inputs.case_seed(1, 0), device=dev)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    ms = timed_sorts(torch, rtcdf, a, b, 0, R, max(steps, 100), stream)
    # Flushed: a 512 MiB write before every sort evicts input and output from
    # the last-level cache; events bracket the sort alone (median of 20).
    scratch = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    flushed = []
    for _ in range(20):
        scratch.fill_(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rtcdf.sort(a, 0, R, keys_out=b, stream=stream)
        e1.record(stream)
        e1.synchronize()
        flushed.append(e0.elapsed_time(e1))
    del scratch
    # The paper's protocol: host wall clock around workspace allocation, the
    # sort and a synchronisation (the library's workspaces are released first).
    wall = []
    for _ in range(10):
        rtcdf.lib.rtcdf_release_workspaces()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rtcdf.sort(a, 0, R, keys_out=b, stream=stream)
        torch.cuda.synchronize()
        wall.append((time.perf_counter() - t0) * 1e3)
    med = lambda v: sorted(v)[len(v) // 2]
    return {"workload": "n=1e6 uniform int32 keys, minVal=0, R=2^7", "ms": round(ms, 5),
            "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 2), "timing": "warm (HIP events, mean)",
            "ms_flushed": round(med(flushed), 5),
            "ms_wall_with_workspace_alloc": round(med(wall), 4)}


def bench_output_methods(torch, rtcdf, inputs, steps):
    """The paper's two output methods on the same inputs and configuration:
    the search of the local CDFs (Alg. 7, the library's path) and step writes
    plus a prefix maximum (Alg. 3, RTCDF_FLAG_OUTPUT_PREFIX_MAX).  Uniform
    keys, n from 10^5 to 10^8, R from 2^7 to 2^22 (the paper saw Alg. 3 win
    at small n and large R), warm, HIP events; both outputs are compared."""
    import numpy as np
    stream = torch.cuda.current_stream()
    old = rtcdf.get_config_mode()
    rtcdf.set_config_mode(rtcdf.CONFIG_DEFAULT)
    rows, same, faster = [], True, []
    try:
        for i, n in enumerate((10 ** 5, 10 ** 6, 10 ** 7, 10 ** 8)):
            for logR in (7, 13, 18, 22):
                R = 1 << logR
                a = inputs.make_device("uniform", n, 0, R, inputs.case_seed(6, 10 * i + logR))
                b = torch.empty_like(a)
                c = torch.empty_like(a)
                lib_cfg = rtcdf.pick_config(n, 0, R)
                search = rtcdf.make_config(lib_cfg.tile_width, lib_cfg.items_per_thread,
                                           lib_cfg.blocks_per_tile)
                pm = rtcdf.make_config(lib_cfg.tile_width, lib_cfg.items_per_thread, lib_cfg.blocks_per_tile,
                                       flags=rtcdf.FLAG_OUTPUT_PREFIX_MAX)
                reps = max(steps, 20)
                t_fill = timed_sorts(torch, rtcdf, a, b, 0, R, reps, stream, config=search)
                t_pmax = timed_sorts(torch, rtcdf, a, c, 0, R, reps, stream, config=pm)
                same = same and bool(torch.equal(b, c))
                if t_pmax < t_fill:
                    faster.append(f"n={n} R=2^{logR}")
                rows.append({"n": n, "R": R, "ms_search": round(t_fill, 5), "ms_prefix_max": round(t_pmax, 5),
                             "prefix_max_over_search": round(t_pmax / t_fill, 3),
                             "library_choice": "prefix_max" if lib_cfg.flags else "search"})
                del a, b, c
    finally:
        rtcdf.set_config_mode(old)
    picked = [r["ms_prefix_max"] if r["library_choice"] == "prefix_max" else r["ms_search"] for r in rows]
    gm = lambda v: float(np.exp(np.mean(np.log(v))))
    return {"rows": rows, "outputs_identical": same, "prefix_max_faster_at": faster,
            "library_choice_over_search_geomean": round(gm([p / r["ms_search"] for p, r in zip(picked, rows)]), 4),
            "timing": "warm, HIP events, mean over repetitions, default-mode kernel configuration for both"}


def bench_wide_ranges(torch, rtcdf, inputs, steps):
    """n = 10^8 uniform, normal (sd R/6), Zipf(1.1) and all-equal keys over
    R = 2^20, 2^22, 2^24 (beyond the paper's ranges; Zipf and all-equal keys
    put nearly every key in one LDS pass): the library's choice (the
    partition by pass from 9 passes on) against the histogram that reads every key once per pass
    (RTCDF_DEV_PARTITION=0), and the LEARNED mode (these ranges lie outside
    the network's trusted range, so its decision is the exhaustive autotune
    of the grid, made once and cached; timed after it), warm, HIP events;
    the outputs are compared."""
    stream = torch.cuda.current_stream()
    rows, same = [], True
    n = 10 ** 8
    reps = max(3, steps // 4)
    try:
        for logR in WIDE_LOG_R:
            R = 1 << logR
            for dist in ("uniform", "normal", "zipf", "all_equal"):
                a = inputs.make_device(dist, n, 0, R, inputs.case_seed(7, logR))
                b = torch.empty_like(a)
                c = torch.empty_like(a)
                info = rtcdf.plan_info(n, 0, R)
                t_lib = timed_sorts(torch, rtcdf, a, b, 0, R, reps, stream)
                os.environ["RTCDF_DEV_PARTITION"] = "0"
                t_multi = timed_sorts(torch, rtcdf, a, c, 0, R, reps, stream)
                os.environ.pop("RTCDF_DEV_PARTITION")
                same = same and bool(torch.equal(b, c))
                row = {"R": R, "dist": dist, "passes": info["passes"],
                       "partition_buckets": info["partition_buckets"], "ms": round(t_lib, 4),
                       "gkeys_per_s": round(n / (t_lib * 1e-3) / 1e9, 1),
                       "ms_every_pass_reads_all_keys": round(t_multi, 4),
                       "speedup": round(t_multi / t_lib, 2)}
                model = os.path.join(ROOT, "paper_2609_00843_amd", "data", "model.bin")
                if os.path.exists(model):
                    old = rtcdf.get_config_mode()
                    try:
                        rtcdf.load_model(model)
                        rtcdf.set_config_mode(rtcdf.CONFIG_LEARNED)
                        rtcdf.clear_pick_cache()
                        rtcdf.pick_config(n, 0, R, keys_in=a)      # the decision, made once
                        point, src = rtcdf.last_pick()
                        c.fill_(0)
                        t_l = timed_sorts(torch, rtcdf, a, c, 0, R, reps, stream)
                        same = same and bool(torch.equal(b, c))
                        row.update({"ms_learned": round(t_l, 4), "learned_point": int(point),
                                    "learned_flags": rtcdf.config_grid()[0][point][3],
                                    "learned_source": PICK_NAMES.get(src, src),
                                    "gain_learned": round(t_lib / t_l, 3)})
                    finally:
                        rtcdf.set_config_mode(old)
                        rtcdf.clear_pick_cache()
                rows.append(row)
                del a, b, c
    finally:
        os.environ.pop("RTCDF_DEV_PARTITION", None)
    return {"workload": "n=1e8 int32 keys, minVal=0, R in {2^20, 2^22, 2^24}, uniform / normal / zipf / all-equal",
            "rows": rows,
            "outputs_identical": same, "timing": "warm, HIP events, mean"}


def bench_key_widths(torch, rtcdf, steps):
    """n = 10^8 keys of 16 and 8 bits (rtcdf_sort_keys): the type's whole
    range and a 2^13-value range for 16-bit keys, uniform; and int64 keys over
    2^16 and 2^18 values at minVal 10^12; warm, HIP events; the roofline is
    2 x key bytes per key at 8 TB/s.  Each output is checked to be
    nondecreasing with the input's value counts (bincount on the GPU)."""
    stream = torch.cuda.current_stream()
    n = 10 ** 8
    rows, ok = [], True
    g = torch.Generator(device="cuda")
    for name, dt, kb, lo, hi in (("int16", torch.int16, 2, -32768, 32768), ("int16", torch.int16, 2, -4096, 4096),
                                 ("uint16", torch.uint16, 2, 0, 65536), ("int8", torch.int8, 1, -128, 128),
                                 ("uint8", torch.uint8, 1, 0, 256), ("int64", torch.int64, 8, 10 ** 12, 10 ** 12 + 65536),
                                 ("int64", torch.int64, 8, 10 ** 12, 10 ** 12 + 262144)):
        g.manual_seed((hi - lo) & 0xffffffff)
        off = lo if dt == torch.int64 else 0
        w = torch.randint(lo - off, hi - off, (n,), generator=g, device="cuda", dtype=torch.int32)
        if dt == torch.int64:
            a = w.to(torch.int64) + off
        else:
            a = w.to(torch.int16).view(torch.uint16) if dt == torch.uint16 else w.to(dt)
        b = torch.empty_like(a)
        for _ in range(3):
            rtcdf.sort_keys(a, lo, hi, keys_out=b, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(steps, 10)
        e0.record(stream)
        for _ in range(reps):
            rtcdf.sort_keys(a, lo, hi, keys_out=b, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        if dt == torch.int64:
            wide = (b - off).to(torch.int32)
        else:
            wide = (b.view(torch.int16).to(torch.int32) & 0xFFFF) if dt == torch.uint16 else b.to(torch.int32)
        ok = ok and bool((wide[1:] >= wide[:-1]).all()) and bool(
            torch.equal(torch.bincount(wide - (lo - off), minlength=hi - lo),
                        torch.bincount(w - (lo - off), minlength=hi - lo)))
        rows.append({"keys": name, "minVal": lo, "maxVal": hi, "ms": round(ms, 4),
                     "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 1),
                     "frac_roofline": round(2 * kb * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)})
        del w, a, b, wide
    return {"workload": "n=1e8 uniform 16-, 8- and 64-bit keys", "rows": rows, "checked": ok,
            "timing": "warm, HIP events, mean"}


def profile_large_n(torch, rtcdf, inputs, steps, warmup, flags=0):
    """Profiling mode: the n = 10^9, R = 2^18 arrays of the scale section
    (uniform, all equal, normal sd R/64), `warmup` then `steps` sorts each,
    one array resident at a time (4 GB in + 4 GB out)."""
    dev = torch.device("cuda:0")
    n, R = 1_000_000_000, 1 << 18
    b = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    cfg = rtcdf.make_config(0, 0, 0, flags=flags) if flags else None
    res = {}
    for dist, sd_div in (("uniform", 6.0), ("all_equal", 6.0), ("normal", 64.0)):
        a = inputs.make_device(dist, n, 0, R, inputs.case_seed(3, int(sd_div)), sd_div=sd_div, device=dev)
        for _ in range(warmup):
            rtcdf.sort(a, 0, R, keys_out=b, stream=stream, config=cfg)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            rtcdf.sort(a, 0, R, keys_out=b, stream=stream, config=cfg)
        e1.record(stream)
        torch.cuda.synchronize()
        res[dist] = e0.elapsed_time(e1) / steps
        log(f"[bench] n=1e9 R=2^18 {dist}: {res[dist]:.3f} ms per sort")
        del a
    print(json.dumps({"ms_per_sort": res}))


def profile_picker(torch, rtcdf, inputs, steps, warmup):
    """Profiling mode: the learned picker's kernels.  Per step, for each of
    four arrays (n = 10^8; R = 2^10, 2^16, 2^18; uniform and normal sd R/6)
    with the shipped model in LEARNED mode: the decision cache is cleared and
    rtcdf_pick_config decides (sketch + network pick, k_pick_spread); then
    one call of rtcdf_mlp_train (forward, gradient and Adam kernels) runs
    `steps` training steps on a 2000 x 34 batch of synthetic features."""
    model = os.path.join(ROOT, "paper_2609_00843_amd", "data", "model.bin")
    dev = torch.device("cuda:0")
    n = 10 ** 8
    arrays = [(inputs.make_device(d, n, 0, 1 << lr, inputs.case_seed(8, lr), device=dev), 1 << lr)
              for lr, d in ((10, "uniform"), (16, "normal"), (18, "uniform"), (18, "normal"))]
    rtcdf.load_model(model)
    old = rtcdf.get_config_mode()
    rtcdf.set_config_mode(rtcdf.CONFIG_LEARNED)
    try:
        for k in range(warmup + steps):
            for a, R in arrays:
                rtcdf.clear_pick_cache()
                rtcdf.pick_config(n, 0, R, keys_in=a)
        torch.cuda.synchronize()
    finally:
        rtcdf.set_config_mode(old)
        rtcdf.clear_pick_cache()
    g = torch.Generator(device=dev)
    g.manual_seed(2609)
    B = 2000
    X = torch.randn((B, rtcdf.MLP_INPUTS), generator=g, device=dev)
    T = torch.randn((B, rtcdf.MLP_OUTPUTS), generator=g, device=dev) * 0.1
    M = torch.ones((B, rtcdf.MLP_OUTPUTS), device=dev)
    P = torch.randn(rtcdf.MLP_PARAMS, generator=g, device=dev) * 0.05
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    rtcdf.mlp_train(P, m, v, 0, X, T, M, steps, 1e-3, ws=rtcdf.mlp_workspace(B, dev))
    torch.cuda.synchronize()
    print(json.dumps({"picks": (warmup + steps) * len(arrays), "train_steps": steps}))


def profile_key_widths(torch, rtcdf, steps, warmup):
    """Profiling mode: the whole-range 16- and 8-bit arrays of bench_key_widths
    and its int64 array over 2^18 values, each sorted once per step."""
    n = 10 ** 8
    g = torch.Generator(device="cuda")
    arrays = []
    for dt, lo, hi in ((torch.int16, -32768, 32768), (torch.uint16, 0, 65536), (torch.int8, -128, 128),
                       (torch.uint8, 0, 256)):
        g.manual_seed(hi - lo)
        w = torch.randint(lo, hi, (n,), generator=g, device="cuda", dtype=torch.int32)
        a = w.to(torch.int16).view(torch.uint16) if dt == torch.uint16 else w.to(dt)
        arrays.append((a, torch.empty_like(a), lo, hi))
        del w
    g.manual_seed(262144)
    w = torch.randint(0, 262144, (n,), generator=g, device="cuda", dtype=torch.int32)
    arrays.append((w.to(torch.int64) + 10 ** 12, torch.empty(n, dtype=torch.int64, device="cuda"), 10 ** 12,
                   10 ** 12 + 262144))
    del w
    stream = torch.cuda.current_stream()

    def step():
        for a, b, lo, hi in arrays:
            rtcdf.sort_keys(a, lo, hi, keys_out=b, stream=stream)

    for _ in range(warmup):
        step()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    log(f"[bench] key widths: {ms:.4f} ms per step of {len(arrays)} arrays")
    # the copy reference of the counter calibration (4 x 10^8 bytes)
    src = torch.empty(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(steps):
        rtcdf.stream_copy(src, dst, stream=stream)
    torch.cuda.synchronize()
    print(json.dumps({"ms_per_step": ms, "keys_per_step": n * len(arrays)}))


def bench_scale(torch, rtcdf, inputs, steps):
    """n = 10^9 keys, minVal 0, R = 2^18: uniform, all equal (87381) and normal
    (mean 2^17, sd 4096).  Element-by-element parity at this size is checked
    by the streaming-verifier tests; here only the time is taken."""
    dev = torch.device("cuda:0")
    n, R = 1_000_000_000, 1 << 18
    b = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    rows = []
    for dist, sd_div in (("uniform", 6.0), ("all_equal", 6.0), ("normal", 64.0)):
        a = inputs.make_device(dist, n, 0, R, inputs.case_seed(3, int(sd_div)), sd_div=sd_div, device=dev)
        torch.cuda.synchronize()
        ms = timed_sorts(torch, rtcdf, a, b, 0, R, max(3, steps // 2), stream)
        info = rtcdf.plan_info(n, 0, R, keys_in=a, keys_out=b)
        rows.append({"dist": dist if dist != "normal" else "normal sd R/64", "ms": round(ms, 4),
                     "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 2),
                     "frac_8B_roofline": round(8.0 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "counter_bits": info["counter_bits"], "hist_passes": info["passes"]})
        log(f"[bench] n=1e9 R=2^18 {dist}: {ms:.3f} ms, {rows[-1]['gkeys_per_s']} Gkeys/s")
        del a
    del b
    torch.cuda.empty_cache()
    return {"workload": "n=1e9 int32 keys, minVal=0, R=2^18", "cases": rows}


WIDE_N = (1 << 32) + (1 << 30)


def _wide_input(torch, n, R, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    a = torch.empty(n, dtype=torch.int32, device="cuda")
    for s in range(0, n, 1 << 28):
        e = min(n, s + (1 << 28))
        a[s:e] = torch.randint(0, R, (e - s,), generator=g, device="cuda", dtype=torch.int32)
    return a


def bench_wide(torch, rtcdf, steps):
    """n = 2^32 + 2^30 int32 keys (per-value counts in 64 bits: three pieces
    and output windows of 2^31, 2^31 and 2^30 keys), uniform over R = 2^16 at
    minVal 0; warm, HIP events, mean.  The output is checked to be
    nondecreasing with the input's value counts (bincount on the GPU, in
    chunks); element-by-element parity at this size is the streaming
    verifier's, in the GPU tests."""
    n, R = WIDE_N, 1 << 16
    stream = torch.cuda.current_stream()
    a = _wide_input(torch, n, R, 4242)
    b = torch.empty_like(a)
    ms = timed_sorts(torch, rtcdf, a, b, 0, R, max(3, min(steps, 10)), stream)
    ca = torch.zeros(R, dtype=torch.int64, device="cuda")
    cb = torch.zeros(R, dtype=torch.int64, device="cuda")
    ok = True
    for s in range(0, n, 1 << 28):
        e = min(n, s + (1 << 28))
        ca += torch.bincount(a[s:e], minlength=R)
        cb += torch.bincount(b[s:e], minlength=R)
        ok = ok and bool((b[s + 1:min(n, e + 1)] >= b[s:min(n, e + 1) - 1]).all())
    ok = ok and bool(torch.equal(ca, cb))
    del a, b
    torch.cuda.empty_cache()
    log(f"[bench] n=2^32+2^30 R=2^16 uniform: {ms:.3f} ms, {n / (ms * 1e-3) / 1e9:.1f} Gkeys/s, checked {ok}")
    return {"workload": "n=2^32+2^30 int32 keys (64-bit counts), minVal=0, R=2^16, uniform",
            "n": n, "ms": round(ms, 4), "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 2),
            "frac_8B_roofline": round(8.0 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "checked": ok,
            "timing": "warm, HIP events, mean"}


def profile_wide(torch, rtcdf, steps, warmup):
    """Profiling mode: the array of bench_wide sorted once per step."""
    n, R = WIDE_N, 1 << 16
    stream = torch.cuda.current_stream()
    a = _wide_input(torch, n, R, 4242)
    b = torch.empty_like(a)
    for _ in range(warmup):
        rtcdf.sort(a, 0, R, keys_out=b, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        rtcdf.sort(a, 0, R, keys_out=b, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    print(json.dumps({"ms_per_step": e0.elapsed_time(e1) / steps, "keys_per_step": n}))


def bench_learned(torch, rtcdf, cases, ins, outs, steps):
    """The learned-tuned form against the plain form (DEFAULT mode, the static
    table), measured end to end in this run:
      sweep      every sweep array sorted per step in LEARNED mode (the first
                 sort of a buffer enqueues the network's pick and uses the
                 static choice, later sorts use the decision) against DEFAULT
                 mode, same buffers, after 2 warm-up steps;
      zipf       n = 10^8 Zipf(1.1) keys over R = 2^16 (skewed keys; the
                 network does not trust such sketches, so the grid is timed
                 exhaustively once for the shape class), same protocol;
      first_call the first LEARNED sort of a fresh buffer (pick enqueued) and a
                 DEFAULT sort, HIP events;
      held_out   the re-timed evaluation (learn.evaluate_retimed: exhaustive
                 timing, the LEARNED decision, static / learned / best each
                 the median of 3 run-medians of 30) on the first 40 arrays of
                 the held-out set with n <= 10^8.
    Only what this run measures is reported; the full 500-array held-out
    evaluation is `learn.py heldout`, a run of its own."""
    import math
    from paper_2609_00843_amd import inputs, learn, tune
    model = os.path.join(ROOT, "paper_2609_00843_amd", "data", "model.bin")
    res = {}
    if not os.path.exists(model):
        res["status"] = "no model file"
        return res
    rtcdf.load_model(model)
    stream = torch.cuda.current_stream()
    old = rtcdf.get_config_mode()
    gm = lambda v: math.exp(sum(map(math.log, v)) / len(v))

    def run(mode, arrays, reps):
        rtcdf.set_config_mode(mode)

        def step():
            for a, b, lo, hi in arrays:
                rtcdf.sort(a, lo, hi, keys_out=b, stream=stream)
        for _ in range(2):
            step()
            torch.cuda.synchronize()
        per = []
        for a, b, lo, hi in arrays:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                rtcdf.sort(a, lo, hi, keys_out=b, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            per.append((e0.elapsed_time(e1) / reps, rtcdf.last_pick()))
        return per

    try:
        rtcdf.clear_pick_cache()
        arrays = [(a, b, MIN_VAL, MIN_VAL + (1 << lr)) for (lr, _), a, b in zip(cases, ins, outs)]
        st = run(rtcdf.CONFIG_DEFAULT, arrays, steps)
        le = run(rtcdf.CONFIG_LEARNED, arrays, steps)
        res["sweep"] = [{"R": 1 << lr, "dist": d, "ms_static": round(s_[0], 5), "ms_learned": round(l_[0], 5),
                         "static_point": s_[1][0], "learned_point": l_[1][0],
                         "learned_source": learn.PICK_NAMES.get(l_[1][1], l_[1][1])}
                        for (lr, d), s_, l_ in zip(cases, st, le)]
        res["sweep_gain_geomean"] = round(gm([s_[0] / l_[0] for s_, l_ in zip(st, le)]), 4)
        # Zipf(1.1) keys at n = 10^8, R = 2^16
        z = inputs.make_device("zipf", N, 0, 1 << 16, inputs.case_seed(8, 0))
        zo = torch.empty_like(z)
        zs = run(rtcdf.CONFIG_DEFAULT, [(z, zo, 0, 1 << 16)], steps)[0]
        zl = run(rtcdf.CONFIG_LEARNED, [(z, zo, 0, 1 << 16)], steps)[0]
        uni = [s_[0] for c, s_ in zip(cases, st) if c == (16, "uniform")]
        res["zipf"] = {"workload": "n=1e8 Zipf(1.1) int32 keys, minVal=0, R=2^16", "ms_static": round(zs[0], 5),
                       "ms_learned": round(zl[0], 5), "gain": round(zs[0] / zl[0], 3),
                       "learned_point": zl[1][0], "learned_source": learn.PICK_NAMES.get(zl[1][1], zl[1][1]),
                       # Zipf keys against uniform keys of the same n and R (DEFAULT mode)
                       "static_over_uniform": round(zs[0] / uni[0], 3) if uni else None,
                       "learned_over_uniform": round(zl[0] / uni[0], 3) if uni else None}
        # the first LEARNED call on a fresh buffer: pick enqueued ahead of the sort
        fresh = inputs.make_device("uniform", N, MIN_VAL, MIN_VAL + (1 << 13), inputs.case_seed(8, 1))
        fo = torch.empty_like(fresh)
        rtcdf.set_config_mode(rtcdf.CONFIG_DEFAULT)
        for _ in range(3):
            rtcdf.sort(fresh, MIN_VAL, MIN_VAL + (1 << 13), keys_out=fo, stream=stream)
        t = {}
        for mode in (rtcdf.CONFIG_DEFAULT, rtcdf.CONFIG_LEARNED):
            rtcdf.set_config_mode(mode)
            rtcdf.clear_pick_cache()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(stream)
            rtcdf.sort(fresh, MIN_VAL, MIN_VAL + (1 << 13), keys_out=fo, stream=stream)
            e1.record(stream)
            host_ms = (time.perf_counter() - t0) * 1e3
            torch.cuda.synchronize()
            t[mode] = (e0.elapsed_time(e1), host_ms, learn.PICK_NAMES.get(rtcdf.last_pick()[1]))
        res["first_call"] = {"workload": "n=1e8 uniform, R=2^13, fresh buffer",
                             "gpu_ms_static": round(t[0][0], 5), "gpu_ms_learned_first": round(t[2][0], 5),
                             "host_call_ms_static": round(t[0][1], 4), "host_call_ms_learned_first": round(t[2][1], 4),
                             "learned_first_source": t[2][2]}
        del z, zo, fresh, fo
        # live re-timed held-out subset
        specs = [s_ for s_ in tune.specs("heldout", 500) if s_["n"] <= 10 ** 8][:40]
        summ, _ = learn.evaluate_retimed(specs, model, log=lambda *a: None)
        res["held_out"] = {"arrays": "first 40 of the held-out set (seed unseen by training) with n <= 1e8",
                           **{k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()
                              if k not in ("by_dist", "by_source")},
                           "by_source": {k: round(v["gain_geomean"], 4) for k, v in summ["by_source"].items()}}
    finally:
        rtcdf.set_config_mode(old)
        rtcdf.clear_pick_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cases", default="", help="comma list like 16:uniform,7:normal (default all)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 1e6-key and 1e9-key timings")
    ap.add_argument("--profile-only", action="store_true",
                    help="only run warmup + timed steps (for rocprofv3 runs)")
    ap.add_argument("--wide-ranges", action="store_true",
                    help="with --profile-only: sort n = 10^8 uniform keys over R = 2^20, 2^22 and 2^24 "
                         "(the partition by pass) instead of the range sweep")
    ap.add_argument("--key-widths", action="store_true",
                    help="with --profile-only: sort n = 10^8 uniform int16, uint16, int8 and uint8 keys "
                         "over their whole ranges instead of the range sweep")
    ap.add_argument("--batched", action="store_true",
                    help="with --profile-only: replay the 4096-array batched workload's graph instead of "
                         "the range sweep")
    ap.add_argument("--large-n", action="store_true",
                    help="with --profile-only: sort the n = 10^9, R = 2^18 arrays (uniform, all equal, "
                         "normal sd R/64) instead of the range sweep")
    ap.add_argument("--picker", action="store_true",
                    help="with --profile-only: run the learned picker's decision and training kernels")
    ap.add_argument("--wide-n", action="store_true",
                    help="with --profile-only: sort n = 2^32 + 2^30 keys (64-bit counts) once per step")
    ap.add_argument("--flags", type=lambda x: int(x, 0), default=0,
                    help="with --profile-only: sort with the static knobs and these option flags "
                         "(e.g. 0x40: 4-bit counters) instead of the library's choice")
    ap.add_argument("--output-method", choices=("search", "prefix_max"), default="search",
                    help="with --profile-only: sort with the prefix-maximum output (Alg. 3) instead "
                         "of the local-CDF search (Alg. 7)")
    args = ap.parse_args()
    if args.output_method != "search" and not args.profile_only:
        ap.error("--output-method prefix_max is a profiling mode; it needs --profile-only")
    if args.wide_ranges and not args.profile_only:
        ap.error("--wide-ranges is a profiling mode; it needs --profile-only")
    if args.key_widths and not args.profile_only:
        ap.error("--key-widths is a profiling mode; it needs --profile-only")
    if (args.large_n or args.picker or args.flags or args.wide_n) and not args.profile_only:
        ap.error("--large-n, --wide-n, --picker and --flags are profiling modes; they need --profile-only")
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the library "
              f"drives one GPU (the sort would shard by one 4R-byte histogram all-reduce)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2609_00843_amd import inputs, rtcdf

    if args.key_widths:
        profile_key_widths(torch, rtcdf, args.steps, args.warmup)
        return
    if args.large_n:
        profile_large_n(torch, rtcdf, inputs, args.steps, args.warmup, args.flags)
        return
    if args.wide_n:
        profile_wide(torch, rtcdf, args.steps, args.warmup)
        return
    if args.picker:
        profile_picker(torch, rtcdf, inputs, args.steps, args.warmup)
        return
    if args.batched:
        if not args.profile_only:
            ap.error("--batched is a profiling mode; it needs --profile-only")
        profile_batched(torch, rtcdf, inputs, args.steps, args.warmup)
        return
    cases = [(lr, d) for lr in LOG_R for d in DISTS]
    if args.wide_ranges:
        cases = [(lr, "uniform") for lr in WIDE_LOG_R]
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

    cfgs = [None] * len(cases)
    if args.flags:
        cfgs = [rtcdf.make_config(0, 0, 0, flags=args.flags)] * len(cases)
    if args.output_method == "prefix_max":
        for i, (lr, _) in enumerate(cases):
            c = rtcdf.pick_config(N, MIN_VAL, MIN_VAL + (1 << lr))
            cfgs[i] = rtcdf.make_config(c.tile_width, c.items_per_thread, c.blocks_per_tile,
                                        flags=rtcdf.FLAG_OUTPUT_PREFIX_MAX)

    def step():
        for (lr, _), a, b, c in zip(cases, ins, outs, cfgs):
            rtcdf.sort(a, MIN_VAL, MIN_VAL + (1 << lr), keys_out=b, stream=stream, config=c)

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
    # Attainable write-only bandwidth (the output stage's traffic): torch's
    # vectorised fill of one output array, timed the same way.
    wr0, wr1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        outs[0].fill_(7)
    wr0.record(stream)
    for _ in range(args.steps):
        outs[0].fill_(7)
    wr1.record(stream)
    torch.cuda.synchronize()
    write_gbs = 4.0 * N / (wr0.elapsed_time(wr1) / args.steps * 1e-3) / 1e9
    log(f"[bench] write-only fill of {4 * N} bytes: {write_gbs:.0f} GB/s")

    # Per-case times (same launches, one case at a time): the paper's protocol,
    # the median of 3 run-medians of 30 sorts (HIP events around each sort)
    # after 10 warm-up sorts.
    from paper_2609_00843_amd import learn
    per_case = []
    for (lr, d), a, b in zip(cases, ins, outs):
        R = 1 << lr
        ms = learn.time_config(torch, rtcdf, a, b, MIN_VAL, MIN_VAL + R, None, warmup=10, reps=30, runs=3)
        cfg = rtcdf.pick_config(N, MIN_VAL, MIN_VAL + R)
        per_case.append({"R": R, "dist": d, "ms": round(ms, 5), "timing": "median of 3 run-medians of 30",
                         "gkeys_per_s": round(N / (ms * 1e-3) / 1e9, 2),
                         "frac_8B_roofline": round(8.0 * N / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "config": list(cfg.as_tuple())})
        log(f"[bench] R=2^{lr:<2d} {d:9s} {ms:.4f} ms  {per_case[-1]['gkeys_per_s']:7.1f} Gkeys/s "
            f"{100 * per_case[-1]['frac_8B_roofline']:.1f}% of 8 B/key roofline")

    # Stage times with HIP events recorded by the library on the sort's stream,
    # case by case, grouped per kernel instantiation (the histogram kernel is
    # compiled separately per counter width), so that every entry can
    # be matched with a rocprofv3 per-kernel average.
    kern_ms, kern_n = {}, {}
    stage_tot = {k: 0.0 for k in rtcdf.STAGES}
    nsorts = 0
    for (lr, d), a, b in zip(cases, ins, outs):
        R = 1 << lr
        info = rtcdf.plan_info(N, MIN_VAL, MIN_VAL + R, keys_in=a, keys_out=b)
        # instantiation names: the key width (4 bytes), the wave-aggregation
        # switch, then the LDS-copies switch (int32 keys keep one copy)
        hist_name = (f"k_hist<{info['items_per_thread']}, {info['counter_bits']}, {info['hist_threads']}, 4, "
                     f"{'true' if info['hist_dedupe'] else 'false'}, false>")
        rtcdf.profile_collect()
        rtcdf.profile_enable(True)
        for _ in range(args.steps):
            rtcdf.sort(a, MIN_VAL, MIN_VAL + R, keys_out=b, stream=stream)
        torch.cuda.synchronize()
        st = rtcdf.profile_collect()
        rtcdf.profile_enable(False)
        nsorts += st["sorts"]
        sparse = "true" if N < 64 * R else "false"   # sparse form below 64 keys per value
        if info["scan_workgroups"] == 0:
            # single-tile fast path: two launches, the output stage reduces and scans
            stages = (("hist", hist_name), ("fill", f"k_fill_small<{sparse}, 4>"))
        else:
            stages = (("hist", hist_name), ("reduce", "k_reduce"), ("tilescan", "k_tilescan"),
                      ("fill", f"k_fill<{sparse}, 4>"))
        for stg, name in stages:
            stage_tot[stg] += st[stg]
            kern_ms[name] = kern_ms.get(name, 0.0) + st[stg]
            kern_n[name] = kern_n.get(name, 0) + st["sorts"]
    stage_ms = {k: v / max(nsorts, 1) for k, v in stage_tot.items()}
    algo_bytes = 4.0 * N        # a histogram launch reads every key once; an output launch writes every key once
    kernels = {}
    for name in kern_ms:
        avg = kern_ms[name] / kern_n[name]
        row = {"launches_per_step": kern_n[name] // args.steps, "avg_launch_ms": round(avg, 5),
               "ms_per_step": round(kern_ms[name] / args.steps, 5)}
        if name.startswith("k_hist") or name.startswith("k_fill"):
            row["achieved_GBps"] = round(algo_bytes / (avg * 1e-3) / 1e9, 1)
            row["frac"] = round(algo_bytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        kernels[name] = row
    dominant = max((k for k in kernels if "achieved_GBps" in kernels[k]), key=lambda k: kernels[k]["ms_per_step"])
    dk = kernels[dominant]
    traffic = load_traffic(dominant)
    roofline = {"bound": "hbm", "kernel": dominant,
                "achieved": dk["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["frac"], "traffic": traffic,
                "algorithmic_bytes_per_launch": algo_bytes,
                "avg_launch_ms": dk["avg_launch_ms"],
                "note": "events bracket each stage on the sort's stream; stage timing adds a few "
                        "microseconds per sort, so per-case totals above are measured without it"}

    # CPU oracle on this host over the same arrays; doubles as a full parity check.
    cpu = None
    cpu_parallel = None
    parity = "not checked"
    if not args.no_cpu_baseline:
        import oracle
        t_cpu, k_cpu, bad, host = 0.0, 0, [], []
        # the multi-threaded CPU counting sort runs on this process's CPU share
        par_threads = len(os.sched_getaffinity(0))
        if os.environ.get("OMP_NUM_THREADS", "").isdigit():
            par_threads = min(par_threads, int(os.environ["OMP_NUM_THREADS"]))
        par_bad, par_used = [], 0
        for (lr, d), a, b in zip(cases, ins, outs):
            R = 1 << lr
            A = a.cpu().numpy()
            t = time.perf_counter()
            B = oracle.sort(A, MIN_VAL, MIN_VAL + R)
            t_cpu += time.perf_counter() - t
            k_cpu += A.size
            if not np.array_equal(b.cpu().numpy(), B):
                bad.append(f"2^{lr}:{d}")
            P, par_used = oracle.parallel_sort(A, MIN_VAL, MIN_VAL + R, par_threads)
            if not np.array_equal(P, B):
                par_bad.append(f"2^{lr}:{d}")
            host.append((A, R))
            del B, P
        parity = "bit-exact on all cases" if not bad else f"MISMATCH in {bad}"
        # further whole passes over the same arrays until about 10 s of CPU work
        passes = 1
        while t_cpu < 10.0:
            for A, R in host:
                t = time.perf_counter()
                oracle.sort(A, MIN_VAL, MIN_VAL + R)
                t_cpu += time.perf_counter() - t
                k_cpu += A.size
            passes += 1
        # multi-threaded CPU counting sort: whole passes until about 3 s
        buf = np.empty(max(A.size for A, _ in host), dtype=np.int32)
        t_par, k_par, par_passes = 0.0, 0, 0
        while t_par < 3.0:
            for A, R in host:
                t = time.perf_counter()
                oracle.parallel_sort(A, MIN_VAL, MIN_VAL + R, par_threads, out=buf[:A.size])
                t_par += time.perf_counter() - t
                k_par += A.size
            par_passes += 1
        del host, buf
        cpu_parallel = {
            "value": round(k_par / t_par / 1e9, 4), "unit": "Gkeys/s", "cores": par_used,
            "kind": "multi-threaded counting sort",
            "parity": "bit-exact vs oracle on all cases" if not par_bad else f"MISMATCH in {par_bad}",
            "sample": f"all {len(cases)} arrays of the sweep, {par_passes} passes ({k_par} keys, "
                      f"{t_par:.1f} s), per-thread histograms + parallel fill, {par_used} threads "
                      f"(process affinity {len(os.sched_getaffinity(0))}, "
                      f"{os.cpu_count()} host CPUs)"}
        log(f"[bench] parallel CPU sort {cpu_parallel['value']} Gkeys/s on {par_used} threads; "
            f"{cpu_parallel['parity']}")
        cpu = {"value": round(k_cpu / t_cpu / 1e9, 4), "unit": "Gkeys/s", "cores": 1,
               "kind": "oracle",
               "sample": f"all {len(cases)} arrays of the sweep at full size, {passes} passes "
                         f"({k_cpu} keys, {t_cpu:.1f} s), plain sequential counting sort, 1 thread, "
                         f"{os.cpu_count()} host cores visible"}
        log(f"[bench] oracle {cpu['value']} Gkeys/s on 1 core; parity: {parity}")

    def section(name, fn):
        # A reported section that fails is recorded in the line; it must not
        # cost the measured sweep its JSON line.
        try:
            return fn()
        except Exception as e:
            import traceback
            traceback.print_exc(file=sys.stderr)
            log(f"[bench] {name} failed: {e!r}")
            return {"error": repr(e)}

    learned = None
    if not args.no_learned:
        log("[bench] learned picker vs static table on the sweep")
        learned = section("learned picker",
                          lambda: bench_learned(torch, rtcdf, cases, ins, outs, max(3, args.steps // 2)))
    batched = None
    if not args.no_batched:
        del ins, outs
        torch.cuda.empty_cache()
        log("[bench] batched workload")
        batched = section("batched", lambda: bench_batched(torch, rtcdf, inputs, args.steps,
                                                           not args.no_cpu_baseline))
        if "error" not in batched:
            log(f"[bench] batched: {batched['gkeys_per_s']} Gkeys/s in one graph launch, "
                f"{batched['speedup_vs_plain_calls']}x plain calls, {batched['speedup_vs_plain_graph']}x "
                f"plain graph; parity {batched['parity']}")

    small = large = wide_n = methods = wide = narrow = None
    if not args.no_extra:
        log("[bench] n=1e6 and n=1e9 timings")
        small = section("n=1e6", lambda: bench_small(torch, rtcdf, inputs, args.steps))
        large = section("n=1e9", lambda: bench_scale(torch, rtcdf, inputs, args.steps))
        wide_n = section("n=2^32+2^30", lambda: bench_wide(torch, rtcdf, args.steps))
        log("[bench] output methods: local-CDF search vs prefix maximum")
        methods = section("output methods", lambda: bench_output_methods(torch, rtcdf, inputs, args.steps))
        if "error" not in methods:
            log(f"[bench] output methods identical: {methods['outputs_identical']}; prefix maximum "
                f"faster at: {methods['prefix_max_faster_at'] or 'none'}")
        log("[bench] 16-, 8- and 64-bit keys")
        narrow = section("key widths", lambda: bench_key_widths(torch, rtcdf, args.steps))
        if "error" not in narrow:
            log("[bench] key widths: " + ", ".join(f"{r['keys']} [{r['minVal']},{r['maxVal']}) "
                                                   f"{r['gkeys_per_s']} Gkeys/s" for r in narrow["rows"])
                + f"; checked: {narrow['checked']}")
        log("[bench] wide ranges: partition by pass")
        wide = section("wide ranges", lambda: bench_wide_ranges(torch, rtcdf, inputs, args.steps))
        if "error" not in wide:
            log("[bench] wide ranges: " + ", ".join(f"2^{r['R'].bit_length() - 1} {r['dist']} {r['ms']} ms "
                                                    f"(x{r['speedup']})" for r in wide["rows"])
                + f"; identical: {wide['outputs_identical']}")

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
        "write_fill_GBps": round(write_gbs, 1),
        "min_frac_8B_roofline_R_le_2^16": round(min(c["frac_8B_roofline"] for c in tgt), 4) if tgt else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_parallel": cpu_parallel,
        "parity": parity,
        "stage_ms_per_sort": {k: round(v, 5) for k, v in stage_ms.items()},
        "kernels": kernels,
        "cases": per_case,
        "batched": batched,
        "learned": learned,
        "small_n": small,
        "output_methods": methods,
        "wide_ranges": wide,
        "key_widths": narrow,
        "large_n": large,
        "wide_n": wide_n,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
