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


def test_learned_sorts_do_not_wait_for_the_pick(r):
    """In LEARNED mode the first sort of a buffer enqueues the network's pick
    and sorts with the static choice (source PENDING, or the decision if the
    pick already finished); once the pick has run the next sort decides, and
    later ones reuse the decision (CACHED).  Every output equals the
    oracle's."""
    if not os.path.exists(MODEL):
        pytest.skip("no shipped model")
    r.load_model(MODEL)
    old = r.get_config_mode()
    decided = (r.PICK_NETWORK, r.PICK_NETWORK_KEPT_STATIC, r.PICK_AUTOTUNED)
    try:
        r.set_config_mode(r.CONFIG_LEARNED)
        r.clear_pick_cache()
        for i, (dist, n, lo, R) in enumerate((("uniform", 30_000_000, -5, 1 << 13),
                                              ("normal", 2_000_000, 0, 1 << 17),
                                              ("all_equal", 5_000_000, 3, 1000))):
            A = inputs.make(dist, n, lo, lo + R, inputs.case_seed(72, i))
            a = torch.from_numpy(A).cuda()
            want = oracle.sort(A, lo, lo + R)
            sources = []
            for k in range(3):
                b = r.sort(a, lo, lo + R)
                sources.append(r.last_pick()[1])
                torch.cuda.synchronize()
                assert np.array_equal(b.cpu().numpy(), want)
            _say(f"learned sort sources {dist}: {sources}")
            assert sources[0] in (r.PICK_PENDING,) + decided, (dist, sources)
            assert sources[1] in decided + (r.PICK_CACHED,), (dist, sources)
            assert sources[2] == r.PICK_CACHED or sources[2] == r.PICK_NETWORK_KEPT_STATIC, (dist, sources)
    finally:
        r.set_config_mode(old)
        r.unload_model()
        r.clear_pick_cache()


def test_learned_host_threads(r):
    """LEARNED mode under four host threads, each on a stream of its own,
    sorting the same four buffers in different orders (so that threads meet
    on one pick-cache entry: a pick in flight, a decision being made by
    another thread, the exhaustive fallback for the Zipf keys, which the
    network does not judge), three rounds each.  Every output equals the
    oracle's, whichever configuration each sort ran with."""
    import threading
    if not os.path.exists(MODEL):
        pytest.skip("no shipped model")
    specs = [("uniform", 2_000_003, -5, 1 << 13), ("zipf", 1_000_001, 0, 1 << 16),
             ("normal", 1_500_000, 3, 5000), ("all_equal", 1_048_576, 0, 200)]
    cases = []
    for i, (dist, n, lo, R) in enumerate(specs):
        A = inputs.make(dist, n, lo, lo + R, inputs.case_seed(73, i))
        cases.append((torch.from_numpy(A).cuda(), lo, lo + R, oracle.sort(A, lo, lo + R)))
    torch.cuda.synchronize()
    r.load_model(MODEL)
    old = r.get_config_mode()
    errors = []

    def work(k):
        try:
            s = torch.cuda.Stream()
            order = [(k + j) % len(cases) for j in range(len(cases))]
            for _ in range(3):
                outs = []
                with torch.cuda.stream(s):
                    for i in order:
                        a, lo, hi, _ = cases[i]
                        outs.append((i, r.sort(a, lo, hi)))
                s.synchronize()
                for i, o in outs:
                    if not np.array_equal(o.cpu().numpy(), cases[i][3]):
                        errors.append((k, i))
        except Exception as e:   # reported by the main thread
            errors.append((k, repr(e)))

    try:
        r.set_config_mode(r.CONFIG_LEARNED)
        r.clear_pick_cache()
        _say("learned mode, four host threads")
        threads = [threading.Thread(target=work, args=(k,)) for k in range(4)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        torch.cuda.synchronize()
    finally:
        r.set_config_mode(old)
        r.unload_model()
        r.clear_pick_cache()
    assert not errors, errors


def test_learned_gain_over_static(r):
    """What the trained network (with its exhaustive fallback for sketches it
    does not trust) gains over the method without it: the first 60 arrays of
    the held-out set (a seed no training or tuning decision saw; Zipf keys
    included) with n <= 10^8, and further held-out Zipf arrays up to 24 of
    them.  Each array is timed with the static choice (DEFAULT mode) and with
    LEARNED mode's decision, as the median of 3 run-medians of 30 sorts after
    10 warm-ups; both outputs equal the oracle's counts.  The geometric-mean
    gain must exceed 1.01 over the first 60 arrays and 1.02 over the Zipf
    arrays (8-bit counters wrap on their hot values).  These floors sit below
    the full held-out evaluation's 1.031 and 1.065 by more than the spread of
    such subsamples from box to box (12 Zipf arrays have measured 1.049)."""
    import math
    from paper_2609_00843_amd import learn, tune
    if not os.path.exists(MODEL):
        pytest.skip("no shipped model")
    held = [s for s in tune.specs("heldout", 500) if s["n"] <= 10 ** 8]
    specs = held[:60]
    nz = sum(s["dist"] == "zipf" for s in specs)
    specs += [s for s in held[60:] if s["dist"] == "zipf"][:max(0, 24 - nz)]
    r.load_model(MODEL)
    old = r.get_config_mode()
    gains, zipf = [], []
    try:
        r.clear_pick_cache()
        for s in specs:
            n, lo = s["n"], s["minVal"]
            hi = lo + s["R"]
            a = inputs.make_device(s["dist"], n, lo, hi, s["seed"], sd_div=s["sd_div"])
            b = torch.empty_like(a)
            r.set_config_mode(r.CONFIG_DEFAULT)
            cs = r.pick_config(n, lo, hi)
            r.set_config_mode(r.CONFIG_LEARNED)
            cl = r.pick_config(n, lo, hi, keys_in=a)
            r.set_config_mode(r.CONFIG_DEFAULT)
            ts = learn.time_config(torch, r, a, b, lo, hi, cs)
            tl = ts if cl.as_tuple() == cs.as_tuple() else learn.time_config(torch, r, a, b, lo, hi, cl)
            cnt = oracle.counts(a.cpu().numpy(), lo, hi)
            v = oracle.StreamingVerifier(cnt, lo)
            v.chunk(b.cpu().numpy())
            v.end(n)
            if len(gains) < 60:
                gains.append(ts / tl)
            if s["dist"] == "zipf":
                zipf.append(ts / tl)
            _say(f"gain n={n} R={s['R']} {s['dist']}: static {ts:.4f} learned {tl:.4f} ms ({ts / tl:.3f})")
            del a, b
    finally:
        r.set_config_mode(old)
        r.unload_model()
        r.clear_pick_cache()
    gm = math.exp(sum(map(math.log, gains)) / len(gains))
    gz = math.exp(sum(map(math.log, zipf)) / len(zipf))
    _say(f"geometric-mean gain {gm:.4f} over {len(gains)} arrays, Zipf {gz:.4f} over {len(zipf)}")
    assert gm > 1.01 and gz > 1.02
