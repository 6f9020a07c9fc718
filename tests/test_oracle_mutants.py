"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that
the oracle's pins catch every one of them.  The planted copy is built in a
temporary directory and loaded through RTCDF_ORACLE_LIB in a child process;
the committed oracle is never modified."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rtcdf_oracle.c")

# (name, original text, planted text); every plant keeps memory accesses in bounds.
MUTANTS = [
    ("output_drops_minVal", "B[p] = (int32_t)(minVal + (int64_t)v);", "B[p] = (int32_t)v;"),
    ("tile_test_inclusive", "if (x >= 0 && (uint64_t)x < w) H[b + (uint64_t)x] += 1;",
     "if (x >= 0 && (uint64_t)x <= w) H[b + (uint64_t)x] += 1;"),
    ("scan_drops_last", "for (uint64_t x = 1; x < w; x++) H[b + x] += H[b + x - 1];",
     "for (uint64_t x = 1; x + 1 < w; x++) H[b + x] += H[b + x - 1];"),
    ("offset_uses_first_bin", "offset += H[b + w - 1];", "offset += H[b];"),
    ("search_strict", "if (C[mid] >= p + 1) hi = mid; else lo = mid + 1;",
     "if (C[mid] > p + 1) hi = mid; else lo = mid + 1;"),
    ("stepwrite_skips_first", "for (uint64_t d = 1; d < R; d++)        /* a step of the CDF at d */",
     "for (uint64_t d = 2; d < R; d++)        /* a step of the CDF at d */"),
    ("prefix_max_late_start", "for (uint64_t i = 1; i < n; i++)        /* inclusive prefix maximum */",
     "for (uint64_t i = 2; i < n; i++)        /* inclusive prefix maximum */"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / f"liboracle_{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC",
                           "-I", os.path.join(ROOT, "oracle"), "-o", str(so), str(mut)])
    env = dict(os.environ, RTCDF_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} passed every pin:\n{r.stdout[-2000:]}"
