"""Seeded synthetic key arrays for the RT-CDF workloads.

This module produces inputs only.  It holds none of the sorting method's
arithmetic, imports neither the HIP binding nor the oracle, and is the one
piece the tests, the benchmark and the oracle's callers share.

Distributions (the paper's evaluation uses synthetic uniform, normal and
all-equal keys, Sec. 4.1 and Sec. 4.2; the parameters below are those of the
measured workloads, which differ from the paper's normal sd of R/8 and
all-zero keys):
  uniform    i.i.d. integers in [minVal, maxVal)
  normal     real N(minVal + R/2, (R/sd_div)^2), rounded half-to-even, clamped
             to [minVal, maxVal - 1]
  all_equal  every key = minVal + floor(R/3)
  zipf       rank r in [1, R] with P(r) proportional to r^(-s); key = minVal + r - 1

Every array is generated in fixed chunks of CHUNK keys, chunk c drawing from a
Philox stream keyed by (seed, c).  Element i therefore depends only on (seed,
i), so a prefix of a long array equals the short array with the same seed, and
chunks can be generated in parallel.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 1 << 22
BASE_SEED = 0x26090843
DISTRIBUTIONS = ("uniform", "normal", "all_equal", "zipf")


def case_seed(config: int, case: int, base: int = BASE_SEED) -> int:
    """A 63-bit seed for case `case` of workload `config`."""
    ss = np.random.SeedSequence([base, config, case])
    return int(ss.generate_state(1, dtype=np.uint64)[0] >> np.uint64(1))


def _rng(seed: int, chunk: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed), int(chunk)])))


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(n: int, seed: int, fill) -> np.ndarray:
    out = np.empty(int(n), dtype=np.int32)
    nchunks = (int(n) + CHUNK - 1) // CHUNK

    def one(c):
        lo = c * CHUNK
        hi = min(int(n), lo + CHUNK)
        out[lo:hi] = fill(_rng(seed, c), hi - lo)

    if nchunks <= 1:
        for c in range(nchunks):
            one(c)
    else:
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(one, range(nchunks)))
    return out


def _check_range(minVal: int, maxVal: int) -> int:
    R = int(maxVal) - int(minVal)
    if R <= 0 or minVal < -(2 ** 31) or maxVal > 2 ** 31:
        raise ValueError(f"bad key range [{minVal}, {maxVal})")
    return R


def uniform(n: int, minVal: int, maxVal: int, seed: int) -> np.ndarray:
    _check_range(minVal, maxVal)
    return _chunked(n, seed, lambda g, k: g.integers(int(minVal), int(maxVal), size=k,
                                                     dtype=np.int64))


def normal(n: int, minVal: int, maxVal: int, seed: int, sd_div: float = 6.0) -> np.ndarray:
    R = _check_range(minVal, maxVal)
    mean = float(minVal) + R / 2.0
    sd = R / float(sd_div)

    def fill(g, k):
        x = np.rint(g.normal(mean, sd, size=k))
        np.clip(x, float(minVal), float(maxVal - 1), out=x)
        return x.astype(np.int64)

    return _chunked(n, seed, fill)


def all_equal(n: int, minVal: int, maxVal: int, seed: int = 0) -> np.ndarray:
    R = _check_range(minVal, maxVal)
    return np.full(int(n), int(minVal) + R // 3, dtype=np.int32)


def zipf(n: int, minVal: int, maxVal: int, seed: int, s: float = 1.1) -> np.ndarray:
    R = _check_range(minVal, maxVal)
    w = np.arange(1, R + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def fill(g, k):
        u = g.random(size=k)
        r = np.searchsorted(cdf, u, side="right")      # rank - 1
        np.minimum(r, R - 1, out=r)
        return int(minVal) + r.astype(np.int64)

    return _chunked(n, seed, fill)


def make(dist: str, n: int, minVal: int, maxVal: int, seed: int, **kw) -> np.ndarray:
    if dist == "uniform":
        return uniform(n, minVal, maxVal, seed)
    if dist == "normal":
        return normal(n, minVal, maxVal, seed, kw.get("sd_div", 6.0))
    if dist in ("all_equal", "equal"):
        return all_equal(n, minVal, maxVal)
    if dist == "zipf":
        return zipf(n, minVal, maxVal, seed, kw.get("s", 1.1))
    raise ValueError(f"unknown distribution {dist!r}")


def batched_segments(num: int = 4096, seed: int = None, n_lo: float = 1e3, n_hi: float = 1e6,
                     r_lo_log2: float = 4.0, r_hi_log2: float = 16.0,
                     min_lo: int = -1_000_000, min_hi: int = 1_000_000):
    """Descriptors of the batched workload: per array, n log-uniform in
    [n_lo, n_hi], minVal uniform in [min_lo, min_hi], R log-uniform in
    [2^r_lo_log2, 2^r_hi_log2] (rounded to an integer), distribution drawn
    uniformly from {uniform, normal sd R/6, all-equal}."""
    if seed is None:
        seed = case_seed(4, 0)
    g = _rng(seed, 0)
    ln = g.uniform(math.log(n_lo), math.log(n_hi), size=num)
    ns = np.rint(np.exp(ln)).astype(np.int64)
    mins = g.integers(min_lo, min_hi + 1, size=num, dtype=np.int64)
    lr = g.uniform(r_lo_log2, r_hi_log2, size=num)
    Rs = np.rint(2.0 ** lr).astype(np.int64)
    dists = g.integers(0, 3, size=num)
    names = ("uniform", "normal", "all_equal")
    segs = []
    for i in range(num):
        segs.append(dict(n=int(ns[i]), minVal=int(mins[i]), maxVal=int(mins[i] + Rs[i]),
                         dist=names[int(dists[i])], seed=int(case_seed(4, 1 + i, seed))))
    return segs


def make_device(dist: str, n: int, minVal: int, maxVal: int, seed: int, device="cuda",
                sd_div: float = 6.0, s: float = 1.1):
    """The same four distributions generated on the GPU with torch's Philox
    generator (seeded), for workloads too large to generate on the host in
    reasonable time.  Returns a contiguous int32 tensor on `device`.  The
    values differ from the host generators' (another generator), so callers
    that compare with the oracle copy these arrays back to the host."""
    import torch
    R = _check_range(minVal, maxVal)
    n = int(n)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & ((1 << 63) - 1))
    out = torch.empty(n, dtype=torch.int32, device=device)
    step = 1 << 26
    if dist == "uniform":
        for lo in range(0, n, step):
            hi = min(n, lo + step)
            out[lo:hi] = torch.randint(int(minVal), int(maxVal), (hi - lo,), generator=g,
                                       device=device, dtype=torch.int64).to(torch.int32)
    elif dist == "normal":
        mean, sd = float(minVal) + R / 2.0, R / float(sd_div)
        for lo in range(0, n, step):
            hi = min(n, lo + step)
            x = torch.randn(hi - lo, generator=g, device=device, dtype=torch.float64)
            x = torch.round(x * sd + mean).clamp_(float(minVal), float(maxVal - 1))
            out[lo:hi] = x.to(torch.int64).to(torch.int32)
    elif dist in ("all_equal", "equal"):
        out.fill_(int(minVal) + R // 3)
    elif dist == "zipf":
        w = torch.arange(1, R + 1, device=device, dtype=torch.float64) ** (-float(s))
        cdf = torch.cumsum(w, 0)
        cdf /= cdf[-1].clone()
        for lo in range(0, n, step):
            hi = min(n, lo + step)
            u = torch.rand(hi - lo, generator=g, device=device, dtype=torch.float64)
            r = torch.searchsorted(cdf, u, right=True).clamp_(max=R - 1)
            out[lo:hi] = (r + int(minVal)).to(torch.int32)
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    return out
