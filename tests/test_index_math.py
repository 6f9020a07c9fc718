"""CPU check of the output stage's position arithmetic near n = 2^32: the
step-end test the output walks use (past_step in rtcdf_device.h), compiled
for the host from the same header the kernels include, agrees with 64-bit
arithmetic for every step start within four steps of 2^32, and the 32-bit
form the walks used before (e <= p + span - 1) is shown to wrap there."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "index_math_check.cpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_step_end_near_2pow32(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "index_math_check")
    subprocess.check_call([HIPCC, "--offload-host-only", "-O2", "-std=c++17", "-o", exe, SRC])
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "wrong 0 " in r.stdout
