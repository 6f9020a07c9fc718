"""Reference for the static default-configuration table -- TEST
INFRASTRUCTURE ONLY.

Sec. 4.1 of the paper selects, for every range size R, the tile width whose
geometric mean of relative times r = t(config, condition) / t_min(condition)
over the measured conditions (input sizes and distributions) is smallest.
This is that rule written out for any configuration key.
"""
from __future__ import annotations

import math


def select_per_range(rows):
    """rows: iterable of (R, condition, config, time).  Returns {R: config}.
    Every config of an R must have been timed under every condition of that
    R.  Ties go to the smallest config (Python ordering)."""
    by_r = {}
    for R, cond, cfg, t in rows:
        by_r.setdefault(R, {}).setdefault(cond, {})[cfg] = float(t)
    out = {}
    for R, conds in by_r.items():
        configs = sorted(next(iter(conds.values())).keys())
        best, best_cfg = None, None
        for cfg in configs:
            log_sum = 0.0
            for cond, times in conds.items():
                tmin = min(times.values())
                log_sum += math.log(times[cfg] / tmin)
            gm = math.exp(log_sum / len(conds))
            if best is None or gm < best:
                best, best_cfg = gm, cfg
        out[R] = best_cfg
    return out


def geomean_ratio(times_a, times_b):
    """Geometric mean of times_a[i] / times_b[i] (the gain of b over a when > 1)."""
    s = 0.0
    for a, b in zip(times_a, times_b):
        s += math.log(a / b)
    return math.exp(s / len(times_a))
