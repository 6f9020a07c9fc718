"""Reader for the small key = value fixtures in tests/golden/."""
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    out = {}
    with open(os.path.join(_HERE, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            vals = [int(x) for x in v.split()]
            out[k] = np.array(vals, dtype=np.int64) if len(vals) != 1 or k in ("A", "B") else vals[0]
    return out
