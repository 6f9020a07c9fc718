"""GPU parity over a seeded random mix of problems: each case draws every axis
at once -- key type (int32, int64, 16- and 8-bit, signed or not), n (1 to
5 x 10^5, and 5 x 10^5 to 4 x 10^6 in the large set), the range R (1 to 2^23
for int32 and int64 keys, 2^25 in the large set; any window of a narrow
type), minVal anywhere in the type (its extremes included), the key
distribution, the input and output offsets inside a 16-byte vector, in place
or not, the configuration (the library's choice, flags alone, or explicit
knobs with any tile width that is a multiple of 128; flags for int32 keys
only, as the boundary requires) and, for int32 keys, the entry point
(rtcdf_sort, rtcdf_sort_with_config, rtcdf_sort_ws, rtcdf_sort_noalloc,
rtcdf_sort_checked).  The structured tests cover each axis on its own; this
one covers their combinations.

Every output is compared element by element with the oracle's sort of the
normalised values (Sec. 2.1: the counting sort over [0, R), minVal added
back), and the words around the output and the input are checked unchanged.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2609_00843_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_CASES = 600
N_LARGE = 120
TYPES = {"int32": (np.int32, -(1 << 31), 1 << 31), "int64": (np.int64, -(1 << 63), (1 << 63) - 1),
         "int16": (np.int16, -32768, 32768), "uint16": (np.uint16, 0, 65536),
         "int8": (np.int8, -128, 128), "uint8": (np.uint8, 0, 256)}


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def r():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_00843_amd import rtcdf
    return rtcdf


def _to_dev(A, npt, pad, fill):
    """Device buffer holding A at element offset pad, `fill` around it."""
    buf = np.full(A.size + pad + 16, fill, dtype=npt)
    buf[pad:pad + A.size] = A
    if npt is np.uint16:
        t = torch.from_numpy(buf.view(np.int16)).cuda().view(torch.uint16)
    else:
        t = torch.from_numpy(buf).cuda()
    return t, t[pad:pad + A.size]


def _to_host(t, npt):
    if npt is np.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def _offsets(rng, dist, n, R, seed):
    """n values in [0, R) (int64) with the named distribution."""
    if dist == "few":
        vals = rng.integers(0, R, size=int(rng.integers(1, 6)))
        return vals[rng.integers(0, vals.size, size=n)].astype(np.int64)
    if dist == "normal64":
        return inputs.make("normal", n, 0, R, seed, sd_div=64.0).astype(np.int64)
    return inputs.make(dist, n, 0, R, seed).astype(np.int64)


def _rand_config(rng, r, int32_keys):
    """None (the library's choice), flags alone, or explicit knobs; the flags
    are offered for int32 keys only (other key types take none)."""
    u = rng.random()
    if u < 0.4:
        return None
    flags = 0
    if rng.random() < 0.3:
        flags |= r.FLAG_OUTPUT_PREFIX_MAX
    flags |= int(rng.choice([0, 0, r.FLAG_COUNTERS_16, r.FLAG_COUNTERS_32, r.FLAG_COUNTERS_4]))
    if rng.random() < 0.25:
        flags |= r.FLAG_WAVE_DEDUPE
    if rng.random() < 0.25:
        flags |= r.FLAG_CHUNK_4096
    if not int32_keys:
        flags = 0
    if u < 0.55 and flags:
        return r.make_config(0, 0, 0, flags)
    bpt = int(rng.choice([1, 2, 4]))
    tiles_max = min(256, 163840 // (4 * bpt) // 128)
    T = 128 * int(rng.integers(1, tiles_max + 1))
    return r.make_config(T, int(rng.choice([4, 8, 16])), bpt, flags)


def _case(k, large=False):
    """Case k's draws; `large`: n from 5 x 10^5 to 4 x 10^6 and R up to 2^25
    (many output chunks and tiles, the partition by pass)."""
    rng = np.random.default_rng(inputs.case_seed(94 if large else 91, k))
    name = str(rng.choice(list(TYPES), p=[0.45, 0.15, 0.1, 0.1, 0.1, 0.1]))
    npt, tlo, thi = TYPES[name]
    if large:
        n = int(round(10 ** rng.uniform(5.7, 6.6)))
    else:
        n = int(rng.integers(1, 24)) if rng.random() < 0.15 else int(round(10 ** rng.uniform(0, 5.7)))
    if name in ("int32", "int64"):
        R = max(1, int(round(2 ** rng.uniform(0, 25 if large else 23))))
        if rng.random() < 0.2:
            R = max(1, (1 << int(rng.integers(0, 23))) + int(rng.integers(-1, 2)))
    else:
        R = int(rng.integers(1, thi - tlo + 1)) if rng.random() < 0.6 else thi - tlo
    u = rng.random()
    if u < 0.15:
        lo = tlo                      # the type's lowest value
    elif u < 0.3:
        lo = thi - R                  # the range ends at the type's top (INT64_MAX excluded)
    elif name == "int64":
        lo = min(max(2 * int(rng.integers(-(1 << 62), 1 << 62)), tlo), thi - R)
    else:
        lo = tlo + int(rng.integers(0, thi - R - tlo + 1))
    dist = str(rng.choice(["uniform", "normal", "normal64", "all_equal", "zipf", "few"]))
    return rng, name, npt, n, lo, R, dist


@pytest.mark.parametrize("k", range(N_CASES))
def test_mixed(r, k):
    _run_case(r, k, False)


@pytest.mark.parametrize("k", range(N_LARGE))
def test_mixed_large(r, k):
    _run_case(r, k, True)


def _run_case(r, k, large):
    rng, name, npt, n, lo, R, dist = _case(k, large)
    hi = lo + R
    off = _offsets(rng, dist, n, R, inputs.case_seed(95 if large else 92, k))
    A = (off + np.int64(lo)).astype(npt) if name != "int64" else off + np.int64(lo)
    kb = np.dtype(npt).itemsize
    pin, pout = int(rng.integers(0, 16 // kb)), int(rng.integers(0, 16 // kb))
    inplace = rng.random() < 0.15
    cfg = _rand_config(rng, r, name == "int32")
    entry = str(rng.choice(["sort", "sort_ws", "noalloc", "checked"])) if name == "int32" else "sort_keys"
    _say(f"mixed{' large' if large else ''} {k}: {name} n={n} [{lo},{hi}) R={R} {dist} pin={pin} pout={pout} inplace={inplace} "
         f"cfg={None if cfg is None else cfg.as_tuple()} entry={entry}")
    want = (oracle.sort(off.astype(np.int32), 0, R).astype(np.int64) + np.int64(lo)).astype(npt)
    bin_, tin = _to_dev(A, npt, pin, 7)
    if inplace:
        bout, tout = bin_, tin
    else:
        bout, tout = _to_dev(np.zeros(n, dtype=npt), npt, pout, 0x5A)
    if entry == "sort_keys":
        r.sort_keys(tin, lo, hi, keys_out=tout, config=cfg)
    elif entry == "sort":
        r.sort(tin, lo, hi, keys_out=tout, config=cfg)
    elif entry == "checked":
        r.sort_checked(tin, lo, hi, keys_out=tout, config=cfg)
    else:
        need = r.workspace_bytes(n, lo, hi, config=cfg, keys_out=tout)
        if entry == "noalloc" and need <= r.NOALLOC_MAX_WORKSPACE:
            r.sort_noalloc(tin, tout, lo, hi, config=cfg)
        else:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
            r.sort_ws(tin, tout, lo, hi, ws, config=cfg)
    torch.cuda.synchronize()
    got = _to_host(tout, npt)
    assert np.array_equal(got, want), f"mismatch at {np.flatnonzero(got != want)[:8]}"
    full = _to_host(bout, npt)
    guard = np.array(7 if inplace else 0x5A, dtype=npt)
    pad = pin if inplace else pout
    assert np.all(full[:pad] == guard) and np.all(full[pad + n:] == guard), "words around the output changed"
    if not inplace:
        assert np.array_equal(_to_host(tin, npt), A), "the input changed"


def _prepare(r, k, seed_base, noalloc=True):
    """Inputs, expected output and call of random case k (from the seed space
    `seed_base`) for enqueueing without a wait: (name, run(stream), check()).
    noalloc=False keeps the allocation-free entry point out (its calls must
    not overlap in time, as calls on several streams may)."""
    rng = np.random.default_rng(inputs.case_seed(seed_base, k))
    _, name, npt, n, lo, R, dist = _case(int(rng.integers(0, 1 << 30)))
    hi = lo + R
    off = _offsets(rng, dist, n, R, inputs.case_seed(seed_base + 1, k))
    A = (off + np.int64(lo)).astype(npt) if name != "int64" else off + np.int64(lo)
    kb = np.dtype(npt).itemsize
    pin, pout = int(rng.integers(0, 16 // kb)), int(rng.integers(0, 16 // kb))
    cfg = _rand_config(rng, r, name == "int32")
    entry = str(rng.choice(["sort", "sort_ws", "noalloc"])) if name == "int32" else "sort_keys"
    if entry == "noalloc" and not noalloc:
        entry = "sort_ws"
    want = (oracle.sort(off.astype(np.int32), 0, R).astype(np.int64) + np.int64(lo)).astype(npt)
    _, tin = _to_dev(A, npt, pin, 7)
    bout, tout = _to_dev(np.zeros(n, dtype=npt), npt, pout, 0x5A)
    ws = None
    if entry in ("sort_ws", "noalloc"):
        need = r.workspace_bytes(n, lo, hi, config=cfg, keys_out=tout)
        if entry == "noalloc" and need > r.NOALLOC_MAX_WORKSPACE:
            entry = "sort_ws"
        if entry == "sort_ws":
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")

    def run(stream):
        if entry == "sort_keys":
            r.sort_keys(tin, lo, hi, keys_out=tout, config=cfg, stream=stream)
        elif entry == "sort":
            r.sort(tin, lo, hi, keys_out=tout, config=cfg, stream=stream)
        elif entry == "noalloc":
            r.sort_noalloc(tin, tout, lo, hi, config=cfg, stream=stream)
        else:
            r.sort_ws(tin, tout, lo, hi, ws, config=cfg, stream=stream)

    def check():
        got = _to_host(tout, npt)
        assert np.array_equal(got, want), (k, name, n, R, entry, np.flatnonzero(got != want)[:5])
        tout.fill_(0)   # the next replay must write it again

    return f"{name} n={n} R={R} {dist} {entry} cfg={None if cfg is None else cfg.as_tuple()}", run, check


@pytest.mark.parametrize("seq", range(4))
def test_random_sequence_one_stream(r, seq):
    """40 random problems enqueued back to back on one stream with no wait
    between them (the state one sort leaves for the next on a stream: the
    fast path's accumulation area and its parity words, carry arrays, the
    workspace growing between two sorts, the allocation-free array), then
    every output checked."""
    cases = [_prepare(r, 40 * seq + i, 97) for i in range(40)]
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    for desc, run, _ in cases:
        _say(f"sequence {seq}: {desc}")
        run(s)
    s.synchronize()
    for _, _, check in cases:
        check()


def test_random_sequence_graph_replays(r):
    """A random sequence of caller-workspace and allocation-free sorts captured
    in one HIP graph and replayed three times, with eager sorts of other
    problems between the replays; every replay's outputs are checked."""
    rng_cases = [_prepare(r, i, 99) for i in range(60)]
    cases = [c for c in rng_cases if "sort_ws" in c[0] or "noalloc" in c[0]][:20]
    others = [c for c in rng_cases if "sort_ws" not in c[0] and "noalloc" not in c[0]][:6]
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    for desc, run, check in cases:   # eager once (and warm-up before capture)
        run(s)
    s.synchronize()
    for _, _, check in cases:
        check()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _, run, _ in cases:
            run(s)
    for rep in range(3):
        _say(f"graph replay {rep} of {len(cases)} sorts")
        g.replay()
        torch.cuda.synchronize()
        for _, _, check in cases:
            check()
        for _, run, check in others:
            run(s)
            s.synchronize()
            check()


@pytest.mark.parametrize("k", range(60))
def test_random_checked(r, k):
    """rtcdf_sort_checked on random int32 problems: in half of them 1 to 3
    keys anywhere in the array (head, body or tail of any alignment) lie
    below minVal or at or above maxVal, down to INT32_MIN and up to
    INT32_MAX; those return KEY_OUT_OF_RANGE with the output untouched, the
    others sort exactly."""
    rng = np.random.default_rng(inputs.case_seed(98, k))
    n = int(round(10 ** rng.uniform(0, 6)))
    R = max(1, int(round(2 ** rng.uniform(0, 20))))
    lo = int(rng.integers(-(1 << 31) + 1, (1 << 31) - R))   # room below and above the range
    off = _offsets(rng, str(rng.choice(["uniform", "normal", "all_equal", "zipf"])), n, R,
                   inputs.case_seed(99, k))
    A = (off + lo).astype(np.int32)
    bad = rng.random() < 0.5
    if bad:
        for _ in range(int(rng.integers(1, 4))):
            i = int(rng.integers(0, n))
            A[i] = int(rng.choice([lo - 1, lo + R, -(1 << 31), (1 << 31) - 1,
                                   int(rng.integers(-(1 << 31), lo)), int(rng.integers(lo + R, 1 << 31))]))
    pin, pout = int(rng.integers(0, 4)), int(rng.integers(0, 4))
    _say(f"checked {k}: n={n} [{lo},{lo + R}) out_of_range={bad} pin={pin} pout={pout}")
    _, tin = _to_dev(A, np.int32, pin, 7)
    bout, tout = _to_dev(np.zeros(n, dtype=np.int32), np.int32, pout, 0x5A)
    if bad:
        with pytest.raises(r.RtcdfError) as e:
            r.sort_checked(tin, lo, lo + R, keys_out=tout)
        assert e.value.status == r.KEY_OUT_OF_RANGE
        torch.cuda.synchronize()
        assert np.all(_to_host(bout, np.int32)[pout:pout + n] == 0), "the output was written"
    else:
        r.sort_checked(tin, lo, lo + R, keys_out=tout)
        torch.cuda.synchronize()
        assert np.array_equal(_to_host(tout, np.int32), oracle.sort(A, lo, lo + R))


def test_random_learned(r):
    """LEARNED mode with the shipped model on 40 random int32 problems (the
    network's picks, the exhaustive fallback for sketches it does not trust,
    each problem sorted twice: the pick in flight, then the decision), and
    rtcdf_autotune on 6 of them (every valid grid point times a sort into
    the output): every output equals the oracle's."""
    import os
    model = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2609_00843_amd",
                         "data", "model.bin")
    if not os.path.exists(model):
        pytest.skip("no shipped model")
    r.load_model(model)
    old = r.get_config_mode()
    try:
        r.set_config_mode(r.CONFIG_LEARNED)
        r.clear_pick_cache()
        for k in range(40):
            rng = np.random.default_rng(inputs.case_seed(100, k))
            n = int(round(10 ** rng.uniform(3, 6.3)))
            R = max(1, int(round(2 ** rng.uniform(0, 22))))
            lo = int(rng.integers(-(1 << 31), (1 << 31) - R + 1))
            dist = str(rng.choice(["uniform", "normal", "normal64", "all_equal", "zipf", "few"]))
            A = (_offsets(rng, dist, n, R, inputs.case_seed(101, k)) + lo).astype(np.int32)
            want = oracle.sort(A, lo, lo + R)
            _, tin = _to_dev(A, np.int32, int(rng.integers(0, 4)), 7)
            _say(f"learned {k}: n={n} [{lo},{lo + R}) {dist}")
            for _ in range(2):
                out = r.sort(tin, lo, lo + R)
                torch.cuda.synchronize()
                assert np.array_equal(out.cpu().numpy(), want), (k, r.last_pick())
            if k % 7 == 0:
                b = torch.empty_like(tin)
                _say(f"autotune {k}")
                times, best = r.autotune(tin, lo, lo + R, keys_out=b, warmup=1, reps=2)
                torch.cuda.synchronize()
                assert np.array_equal(b.cpu().numpy(), want)
                assert min(t for t in times if t > 0) > 0
    finally:
        r.set_config_mode(old)
        r.unload_model()
        r.clear_pick_cache()


def test_random_sequence_three_streams(r):
    """60 random problems dealt round-robin to three streams and enqueued
    with no wait (each stream's cached workspace, fast-path area and carry
    array serve only its own sorts, whatever the others run meanwhile); every
    output checked once all streams are done."""
    cases = [_prepare(r, i, 102, noalloc=False) for i in range(60)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    torch.cuda.synchronize()
    for i, (desc, run, _) in enumerate(cases):
        _say(f"three streams, case {i} on stream {i % 3}: {desc}")
        run(streams[i % 3])
    torch.cuda.synchronize()
    for _, _, check in cases:
        check()


@pytest.mark.parametrize("k", range(100))
def test_random_partition_forced(r, k, monkeypatch):
    """The partition by pass forced on (RTCDF_DEV_PARTITION=1: wherever a
    sort needs two or more LDS passes) for random int32 problems over R from
    2^14 to 2^24 with random configurations, offsets, in place or not, through
    rtcdf_sort and rtcdf_sort_ws: the keys grouped by pass into the
    workspace, each pass's rows counted over its own bucket."""
    monkeypatch.setenv("RTCDF_DEV_PARTITION", "1")
    rng = np.random.default_rng(inputs.case_seed(103, k))
    n = int(round(10 ** rng.uniform(0, 6.3)))
    R = int(round(2 ** rng.uniform(14, 24)))
    u = rng.random()
    lo = -(1 << 31) if u < 0.1 else ((1 << 31) - R if u < 0.2 else int(rng.integers(-(1 << 31), (1 << 31) - R + 1)))
    dist = str(rng.choice(["uniform", "normal", "normal64", "all_equal", "zipf", "few"]))
    off = _offsets(rng, dist, n, R, inputs.case_seed(104, k))
    A = (off + lo).astype(np.int32)
    pin, pout = int(rng.integers(0, 4)), int(rng.integers(0, 4))
    inplace = rng.random() < 0.15
    cfg = _rand_config(rng, r, True)
    entry = str(rng.choice(["sort", "sort_ws"]))
    _say(f"partition forced {k}: n={n} [{lo},{lo + R}) {dist} pin={pin} pout={pout} inplace={inplace} "
         f"cfg={None if cfg is None else cfg.as_tuple()} entry={entry}")
    want = oracle.sort(A, lo, lo + R)
    bin_, tin = _to_dev(A, np.int32, pin, 7)
    tout = tin if inplace else _to_dev(np.zeros(n, dtype=np.int32), np.int32, pout, 0x5A)[1]
    if entry == "sort":
        r.sort(tin, lo, lo + R, keys_out=tout, config=cfg)
    else:
        ws = torch.empty(max(r.workspace_bytes(n, lo, lo + R, config=cfg, keys_out=tout), 256),
                         dtype=torch.uint8, device="cuda")
        r.sort_ws(tin, tout, lo, lo + R, ws, config=cfg)
    torch.cuda.synchronize()
    got = _to_host(tout, np.int32)
    assert np.array_equal(got, want), f"mismatch at {np.flatnonzero(got != want)[:8]}"


DEV_SWITCHES = {"RTCDF_DEV_COUNTER_BITS": ["4", "8", "16", "32"], "RTCDF_DEV_FAST": ["0", "1"],
                "RTCDF_DEV_HIST_SPREAD": ["0", "1", "2", "4"], "RTCDF_DEV_PARTITION": ["0", "1"],
                "RTCDF_DEV_HIST_INTERLEAVE": ["0", "1"], "RTCDF_DEV_FILL_CHUNK": ["2048", "4096", "8192"],
                "RTCDF_DEV_FILL_SPARSE_KEYS": ["16", "64", "256"], "RTCDF_DEV_FAST_ROWS": ["1", "4", "16"],
                "RTCDF_DEV_HIST_GMUL": ["1", "2", "4"], "RTCDF_DEV_PART_WGS_PER_CU": ["2", "4", "8"],
                "RTCDF_DEV_FILL_WGS_PER_CU": ["2", "3", "4", "8"]}


@pytest.mark.parametrize("k", range(120))
def test_random_dev_switches(r, k, monkeypatch):
    """Random problems (every key type) with a random subset of the developer
    overrides set, each to a value the measurements swept (counter width,
    fast path, LDS counter copies, partition by pass, input interleave, output
    chunk, sparse-form threshold, fast-path rows, histogram and partition and
    output workgroups): they change launch shapes only, so every output must
    still equal the oracle's."""
    rng = np.random.default_rng(inputs.case_seed(105, k))
    chosen = {}
    for name, values in DEV_SWITCHES.items():
        if rng.random() < 0.35:
            chosen[name] = str(rng.choice(values))
            monkeypatch.setenv(name, chosen[name])
    _say(f"developer switches {k}: {chosen}")
    _run_case(r, 20000 + k, bool(rng.random() < 0.2))


@pytest.mark.parametrize("k", range(40))
def test_random_workspace_contract(r, k):
    """rtcdf_workspace_bytes on random int32 problems, configurations and
    input / output offsets: a caller workspace of exactly that many bytes
    sorts (into an output at the offset the size was asked for, from an
    input at any offset), one byte less is refused before any GPU work with
    the output untouched."""
    rng = np.random.default_rng(inputs.case_seed(110, k))
    n = int(round(10 ** rng.uniform(0, 6.3)))
    R = max(1, int(round(2 ** rng.uniform(0, 24))))
    lo = int(rng.integers(-(1 << 31), (1 << 31) - R + 1))
    off = _offsets(rng, str(rng.choice(["uniform", "normal", "all_equal", "zipf"])), n, R, inputs.case_seed(111, k))
    A = (off + lo).astype(np.int32)
    cfg = _rand_config(rng, r, True)
    pin, pout = int(rng.integers(0, 4)), int(rng.integers(0, 4))
    _, tin = _to_dev(A, np.int32, pin, 7)
    bout, tout = _to_dev(np.zeros(n, dtype=np.int32), np.int32, pout, 0x5A)
    need = r.workspace_bytes(n, lo, lo + R, config=cfg, keys_out=tout)
    _say(f"workspace contract {k}: n={n} R={R} cfg={None if cfg is None else cfg.as_tuple()} "
         f"pin={pin} pout={pout} bytes={need}")
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    if need > 0:
        with pytest.raises(r.RtcdfError) as e:
            r.sort_ws(tin, tout, lo, lo + R, ws[:need - 1], config=cfg)
        assert e.value.status == r.WORKSPACE_TOO_SMALL
        torch.cuda.synchronize()
        assert np.all(_to_host(tout, np.int32) == 0)
    r.sort_ws(tin, tout, lo, lo + R, ws[:need], config=cfg)
    torch.cuda.synchronize()
    assert np.array_equal(_to_host(tout, np.int32), oracle.sort(A, lo, lo + R))
