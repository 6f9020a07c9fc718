"""GPU tests of the configuration sources: the exhaustive autotuner
(rtcdf_autotune) and sorts in LEARNED mode with the shipped model, each
checked element by element against the oracle (the configuration may change
the speed of a sort, never its output)."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2609_00843_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL = os.path.join(ROOT, "paper_2609_00843_amd", "data", "model.bin")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def r():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_00843_amd import rtcdf
    return rtcdf


@pytest.mark.parametrize("dist,n,lo,R", [("uniform", 200_003, -50, 1000), ("normal", 150_000, 7, 70_000),
                                         ("zipf", 100_001, 0, 300)])
def test_autotune(r, dist, n, lo, R):
    """Every valid grid point gets a positive median time, every invalid one
    -1; the returned best is the argmin of the returned times; the output
    buffer holds the sorted keys (every timed sort writes them)."""
    A = inputs.make(dist, n, lo, lo + R, inputs.case_seed(70, n))
    a = torch.from_numpy(A).cuda()
    b = torch.empty_like(a)
    _say(f"autotune {dist} n={n} R={R}")
    times, best = r.autotune(a, lo, lo + R, keys_out=b, warmup=1, reps=3)
    torch.cuda.synchronize()
    pts, valid = r.config_grid()
    assert len(times) == len(pts) == r.GRID_SIZE
    for t, v in zip(times, valid):
        assert (t > 0) if v else (t == -1.0)
    i = min(range(len(times)), key=lambda j: (times[j] if valid[j] else float("inf"), j))
    assert best.as_tuple() == pts[i]
    assert np.array_equal(b.cpu().numpy(), oracle.sort(A, lo, lo + R))


def test_learned_mode_sorts_match_oracle(r):
    """LEARNED mode with the shipped model: the network's pick (whatever it
    is) sorts every array exactly as the oracle does."""
    if not os.path.exists(MODEL):
        pytest.skip("no shipped model")
    r.load_model(MODEL)
    old = r.get_config_mode()
    try:
        r.set_config_mode(r.CONFIG_LEARNED)
        for i, (dist, n, lo, R) in enumerate((("uniform", 2_000_003, 0, 1 << 17), ("normal", 1_500_000, -3, 5000),
                                              ("zipf", 3_000_001, 11, 1 << 16), ("all_equal", 1_048_576, 0, 200),
                                              ("normal", 4_000_000, 100, 1 << 18))):
            A = inputs.make(dist, n, lo, lo + R, inputs.case_seed(71, i))
            a = torch.from_numpy(A).cuda()
            cfg = r.pick_config(n, lo, lo + R, keys_in=a)
            _say(f"learned {dist} n={n} R={R} -> {cfg}")
            b = r.sort(a, lo, lo + R)
            torch.cuda.synchronize()
            assert np.array_equal(b.cpu().numpy(), oracle.sort(A, lo, lo + R))
    finally:
        r.set_config_mode(old)
        r.unload_model()
