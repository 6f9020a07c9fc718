"""GPU parity of the plain RT-CDF sort against the CPU oracle.

Every comparison is element by element (the output of an unstable sort of bare
integers is unique).  Inputs are seeded; each test prints its case before the
GPU work so a failing run names it.
"""
import itertools
import sys

import numpy as np
import pytest

import oracle
from paper_2609_00843_amd import inputs
from tests.golden.load import load

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def r():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_00843_amd import rtcdf
    return rtcdf


def _to_dev(A, pad_front=0):
    """Device int32 copy of A starting `pad_front` elements into its buffer
    (pad_front in 0..3 makes the array 4/8/12 bytes off 16-byte alignment)."""
    buf = torch.empty(A.size + pad_front + 4, dtype=torch.int32, device="cuda")
    buf.fill_(-12345)
    t = buf[pad_front:pad_front + A.size]
    t.copy_(torch.from_numpy(np.ascontiguousarray(A, dtype=np.int32)))
    return buf, t


def _run(r, A, minVal, maxVal, cfg=None, pin=0, pout=0, inplace=False):
    _say(f"n={A.size} min={minVal} max={maxVal} cfg={cfg} pin={pin} pout={pout} inplace={inplace}")
    want = oracle.sort(A, minVal, maxVal)
    bin_, tin = _to_dev(A, pin)
    if inplace:
        bout, tout = bin_, tin
    else:
        bout = torch.empty(A.size + pout + 8, dtype=torch.int32, device="cuda")
        bout.fill_(0x5A5A5A5A)
        tout = bout[pout:pout + A.size]
    r.sort(tin, minVal, maxVal, keys_out=tout, config=cfg)
    torch.cuda.synchronize()
    got = tout.cpu().numpy()
    assert np.array_equal(got, want), f"mismatch at {np.flatnonzero(got != want)[:8]}"
    if not inplace:
        # guard words around the output are untouched
        full = bout.cpu().numpy()
        assert np.all(full[:pout] == 0x5A5A5A5A) and np.all(full[pout + A.size:] == 0x5A5A5A5A)
        # the input is not modified
        assert np.array_equal(tin.cpu().numpy(), np.asarray(A, dtype=np.int32))


def test_worked_example(r):
    g = load("worked_example.txt")
    _run(r, g["A"].astype(np.int32), g["minVal"], g["maxVal"], r.make_config(128, 4, 1))


def test_small_workload_uniform_1e6(r):
    """n = 10^6 keys, minVal 0, R = 2^7, uniform: the small single-array workload."""
    A = inputs.uniform(10 ** 6, 0, 128, inputs.case_seed(1, 0))
    _run(r, A, 0, 128)


@pytest.mark.parametrize("R", [1, 2, 3, 127, 128, 129, 1000, 4097, 40961, 65535, 65536, 65537,
                               81921, 262144])
def test_ragged_sizes(r, R):
    rng = np.random.default_rng(R)
    for n in (1, 2, 3, 4, 5, 7, 8, 9, 17, 1023, 1025, 4099, 65537, 300001):
        minVal = int(rng.integers(-10 ** 6, 10 ** 6))
        A = rng.integers(minVal, minVal + R, size=n).astype(np.int32)
        _run(r, A, minVal, minVal + R)


@pytest.mark.parametrize("pin,pout", list(itertools.product(range(4), range(4))))
def test_misaligned_pointers(r, pin, pout):
    rng = np.random.default_rng(10 * pin + pout)
    # fast path (sparse and dense), staged 32-bit, one-pass 8-bit
    for n, R in ((13, 50), (300001, 1500), (5000, 3000), (70001, 70000)):
        A = rng.integers(-7, -7 + R, size=n).astype(np.int32)
        _run(r, A, -7, -7 + R, pin=pin, pout=pout)


@pytest.mark.parametrize("R", [128, 70000])
def test_in_place(r, R):
    A = inputs.uniform(123457, 5, 5 + R, 3)
    _run(r, A, 5, 5 + R, inplace=True)
    _run(r, A, 5, 5 + R, pin=1, inplace=True)


@pytest.mark.parametrize("dist", ["uniform", "normal", "all_equal", "zipf"])
@pytest.mark.parametrize("logR", [7, 10, 13, 16, 18])
def test_distributions(r, dist, logR):
    R, minVal = 1 << logR, -1000
    A = inputs.make(dist, 2_000_003, minVal, minVal + R, inputs.case_seed(2, logR))
    _run(r, A, minVal, minVal + R)


@pytest.mark.parametrize("logR,dist", [(20, "normal"), (20, "all_equal"), (21, "uniform"),
                                       (21, "all_equal"), (22, "zipf"), (24, "normal")])
def test_wide_ranges(r, logR, dist):
    """Ranges with up to 1024 tiles and 8192 block totals (the local-CDF stage
    assigns its workgroups by chunk counts) and beyond (fixed split), at the
    default tile width."""
    R = 1 << logR
    A = inputs.make(dist, 3_000_001, -R // 2, R - R // 2, inputs.case_seed(5, logR))
    info = r.plan_info(A.size, -R // 2, R - R // 2)
    assert info["tiles"] == (R + info["tile_width"] - 1) // info["tile_width"]
    _run(r, A, -R // 2, R - R // 2)


def test_extreme_ranges(r):
    i32min = -(2 ** 31)
    A = inputs.uniform(100_001, i32min, i32min + 1000, 1)
    _run(r, A, i32min, i32min + 1000)
    A = inputs.uniform(100_001, 2 ** 31 - 70000, 2 ** 31, 2)
    _run(r, A, 2 ** 31 - 70000, 2 ** 31)
    A = np.full(1000, 2 ** 31 - 1, dtype=np.int32)
    _run(r, A, 2 ** 31 - 1, 2 ** 31)


@pytest.mark.parametrize("R", [1 << 16, 1 << 16 | 1, 81921, 1 << 17, 1 << 18])
def test_packed_counter_overflow(r, R):
    """More equal keys per workgroup than an 8-bit LDS counter holds (255), in
    every byte of one LDS word and in the last bin, with the counter width the
    plan chooses (8-bit for all of these ranges); 16-bit counters are covered
    by the forced-width test below and by the batched sort."""
    n = 40_000_000
    rng = np.random.default_rng(R)
    for pick in ([0], [0, 1], [1], [R - 1], [2, 3, R - 1], [0, 1, 2, 3], [4, 6, 7]):
        vals = np.asarray(pick, dtype=np.int64)
        A = (vals[rng.integers(0, vals.size, size=n)] - 77).astype(np.int32)
        _run(r, A, -77, -77 + R)


@pytest.mark.parametrize("k", [97, 1024, 20000])
def test_few_distinct_values_wide_range(r, k):
    """k distinct values spread over R = 2^18: each of them wraps 8-bit
    counters a few times (k = 97, 1024) or about once (k = 20000) per
    workgroup."""
    R = 1 << 18
    rng = np.random.default_rng(k)
    vals = rng.choice(R, size=k, replace=False)
    A = vals[rng.integers(0, k, size=20_000_000)].astype(np.int32)
    _run(r, A, 0, R)


@pytest.mark.parametrize("R", [1 << 16, (1 << 18) + 5, 1 << 20])
def test_nibble_counter_overflow(r, R):
    """4-bit counters (RTCDF_FLAG_COUNTERS_4): more equal keys per workgroup
    than a nibble holds (15), in every nibble of one LDS word, across words
    and in the last bin; and few distinct values spread over the range."""
    n = 6_000_001
    rng = np.random.default_rng(R + 4)
    cfg = r.make_config(0, 0, 0, flags=r.FLAG_COUNTERS_4)
    assert r.plan_info(n, -77, -77 + R, config=cfg)["counter_bits"] == 4
    picks = ([0], [0, 1], [7], [R - 1], [2, 3, R - 1], list(range(8)), [5, 8, 9, 15, 16])
    for pick in list(picks) + [list(rng.choice(R, size=300, replace=False))]:
        vals = np.asarray(pick, dtype=np.int64)
        A = (vals[rng.integers(0, vals.size, size=n)] - 77).astype(np.int32)
        _say(f"nibble overflow R={R} values={len(pick)}")
        _run(r, A, -77, -77 + R, cfg=cfg)


@pytest.mark.parametrize("bits", [4, 8, 16, 32])
@pytest.mark.parametrize("dist,R", [("zipf", 1000), ("normal", 65537), ("uniform", 1 << 18),
                                    ("all_equal", 1 << 17)])
def test_forced_counter_width(r, monkeypatch, bits, dist, R):
    """Every counter width gives the same output on every range, whichever the
    plan would choose by itself."""
    monkeypatch.setenv("RTCDF_DEV_COUNTER_BITS", str(bits))
    A = inputs.make(dist, 3_000_017, 9, 9 + R, inputs.case_seed(4, R))
    info = r.plan_info(A.size, 9, 9 + R)
    assert info["counter_bits"] == bits
    _run(r, A, 9, 9 + R)


@pytest.mark.parametrize("sub", [1, 4])
@pytest.mark.parametrize("fast", [1, 0])
@pytest.mark.parametrize("dist,R", [("uniform", 100), ("all_equal", 2048), ("zipf", 1500), ("normal", 5000)])
def test_counter_copies(r, monkeypatch, sub, fast, dist, R):
    """LDS copies of the 32-bit counters (2^sub per bin, lane-selected, summed
    when written out) give the same output on the single-tile fast path (the
    merge rows) and the staged path (partial rows), ragged n, input and output
    off their 16-byte alignment."""
    monkeypatch.setenv("RTCDF_DEV_HIST_SPREAD", str(sub))
    monkeypatch.setenv("RTCDF_DEV_FAST", str(fast))
    A = inputs.make(dist, 1_000_003, -5, -5 + R, inputs.case_seed(5, R))
    _run(r, A, -5, -5 + R, pin=1, pout=2)


def test_plan_counter_width_choice(r):
    """The plan takes 32-bit counters where they need no more passes, else
    8-bit ones."""
    widths = {R: r.plan_info(10 ** 8, 0, R)["counter_bits"] for R in (128, 65536, 1 << 17, 1 << 18)}
    assert widths[128] == 32 and widths[65536] == 8
    assert widths[1 << 17] == 8 and widths[1 << 18] == 8


def _grid():
    for T in (1024, 2048, 4096, 8192, 16384, 32768):
        for items in (4, 8, 16):
            for bpt in (1, 2, 4):
                if T * 4 * bpt <= 163840:
                    yield T, items, bpt


GRID = list(_grid())


def test_grid_has_45_valid_points():
    assert len(GRID) == 45


@pytest.mark.parametrize("dist,logR", [("uniform", 7), ("normal", 13), ("all_equal", 16),
                                       ("uniform", 16), ("normal", 18)])
def test_every_config_is_identical(r, dist, logR):
    R, minVal = 1 << logR, 321
    A = inputs.make(dist, 777_777, minVal, minVal + R, inputs.case_seed(5, logR))
    want = oracle.sort(A, minVal, minVal + R)
    _, tin = _to_dev(A, 1)
    for T, items, bpt in GRID:
        _say(f"config T={T} items={items} bpt={bpt} dist={dist} R={R}")
        out = r.sort(tin, minVal, minVal + R, config=r.make_config(T, items, bpt))
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want), (T, items, bpt)


OPTION_FLAGS = (0x01, 0x04, 0x14, 0x10, 0x20, 0x24, 0x08, 0x18, 0x30, 0x11, 0x15, 0x40, 0x50, 0x60, 0x41)


@pytest.mark.parametrize("dist,n,logR", [("uniform", 777_777, 7), ("zipf", 1_000_003, 10), ("normal", 2_000_001, 13),
                                         ("zipf", 3_000_000, 16), ("all_equal", 500_000, 16),
                                         ("normal", 1_500_001, 18), ("zipf", 999_999, 18)])
def test_option_flags_are_identical(r, dist, n, logR):
    """Every option flag (counter widths, wave aggregation of duplicates,
    4096-position chunks, the prefix-maximum output) and some combinations,
    on the static knobs and on explicit ones, give the oracle's output."""
    R, minVal = 1 << logR, -77
    A = inputs.make(dist, n, minVal, minVal + R, inputs.case_seed(6, logR * 7 + n % 5))
    want = oracle.sort(A, minVal, minVal + R)
    _, tin = _to_dev(A, 2)
    for flags in OPTION_FLAGS:
        for cfg in (r.make_config(0, 0, 0, flags=flags), r.make_config(2048, 8, 2, flags=flags)):
            _say(f"option flags {flags:#x} cfg={cfg} {dist} R={R}")
            out = r.sort(tin, minVal, minVal + R, config=cfg)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), want), (flags, cfg)
    info = r.plan_info(n, minVal, minVal + R, config=r.make_config(0, 0, 0, flags=0x14))
    assert info["counter_bits"] == 16 and info["hist_dedupe"] == 1
    info = r.plan_info(n, minVal, minVal + R, config=r.make_config(0, 0, 0, flags=0x40))
    assert info["counter_bits"] == 4


@pytest.mark.parametrize("R,T", [(4, 128), (1000, 128), (1000, 1024), (70000, 1024),
                                 (70000, 32768), (262144, 8192), (300000, 32768),
                                 ((1 << 21) + 77, 128),    # 16385 tiles: offsets by k_tile_offsets
                                 # tile widths that are multiples of 128 but not powers of two:
                                 # 111, 96, 37 and 129 block totals of 128 bins per tile
                                 (1005816, 14208), (300000, 12288), (70000, 4736), (2_000_003, 16512)])
def test_intermediates_match_oracle(r, R, T):
    """Tile histograms (Alg. 5), local CDFs (Alg. 4) and tile offsets (Alg. 6)."""
    rng = np.random.default_rng(R + T)
    minVal = -55
    A = rng.integers(minVal, minVal + R, size=250_000).astype(np.int32)
    A[:1000] = minVal + R - 1
    Teff = min(T, (R + 127) // 128 * 128)
    _say(f"intermediates R={R} T={T} Teff={Teff}")
    h, c, O = oracle.tile_intermediates(A, minVal, minVal + R, Teff)
    _, tin = _to_dev(A, 0)
    gh, gc, gO = r.debug_intermediates(tin, minVal, minVal + R, r.make_config(T, 16, 1))
    torch.cuda.synchronize()
    as_u = lambda t: t.cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal(as_u(gh), h)
    assert np.array_equal(as_u(gc), c)
    assert np.array_equal(as_u(gO), O)


@pytest.mark.parametrize("T,items,bpt", [(14208, 4, 1), (12288, 8, 2), (4736, 16, 4), (16512, 16, 1),
                                         (128 * 255, 4, 1)])
def test_tile_widths_not_powers_of_two(r, T, items, bpt):
    """Any multiple of 128 is a valid tile width: explicit configurations whose
    tiles hold a number of 128-bin blocks that is not a power of two (tile
    boundaries inside a wave's 64 block totals), with the flags that change
    the counters and the output, over several tiles and distributions."""
    for dist, n, R in (("uniform", 121_774, 1_005_816), ("normal", 400_001, 300_000),
                       ("zipf", 250_000, 70_000), ("all_equal", 100_000, 2 * T + 5)):
        A = inputs.make(dist, n, -987, -987 + R, inputs.case_seed(93, T + R))
        want = oracle.sort(A, -987, -987 + R)
        _, tin = _to_dev(A, 1)
        for flags in (0, 0x10, 0x04, 0x01, 0x20):
            cfg = r.make_config(T, items, bpt, flags)
            _say(f"tile width T={T} {dist} n={n} R={R} flags={flags:#x}")
            out = r.sort(tin, -987, -987 + R, config=cfg)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert np.array_equal(got, want), (T, dist, flags, np.flatnonzero(got != want)[:5])


def test_caller_workspace(r):
    rng = np.random.default_rng(9)
    for R in (100, 65536, 200000):
        A = rng.integers(0, R, size=500_001).astype(np.int32)
        want = oracle.sort(A, 0, R)
        _, tin = _to_dev(A, 2)
        out = torch.empty_like(tin)
        nb = r.workspace_bytes(A.size, 0, R, keys_out=out)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        ws.fill_(0xAB)   # contents must not matter
        _say(f"sort_ws R={R} bytes={nb}")
        for _ in range(2):
            r.sort_ws(tin, out, 0, R, ws)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), want)
        with pytest.raises(r.RtcdfError) as e:
            r.sort_ws(tin, out, 0, R, ws[: nb // 2])
        assert e.value.status == r.WORKSPACE_TOO_SMALL


def test_two_streams(r):
    A = inputs.uniform(1_000_000, 0, 70000, 4)
    B = inputs.normal(1_000_000, 0, 300, 5)
    wa, wb = oracle.sort(A, 0, 70000), oracle.sort(B, 0, 300)
    _, ta = _to_dev(A)
    _, tb = _to_dev(B)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    _say("two streams")
    for _ in range(3):
        with torch.cuda.stream(s1):
            oa = r.sort(ta, 0, 70000)
        with torch.cuda.stream(s2):
            ob = r.sort(tb, 0, 300)
        torch.cuda.synchronize()
        assert np.array_equal(oa.cpu().numpy(), wa)
        assert np.array_equal(ob.cpu().numpy(), wb)


def test_host_threads(r):
    """Four host threads, each sorting on a stream of its own (the library's
    per-(device, stream) workspaces and fast-path areas, and its device and
    kernel-attribute caches, under concurrent calls; the binding releases
    the interpreter lock in every library call): the single-tile fast path,
    the staged path with 8-bit counters, two LDS passes and the partition by
    pass, each thread in its own order, three rounds.  Every output equals
    the oracle's."""
    import threading
    specs = [("uniform", 1_000_003, 0, 1000, 11), ("normal", 2_000_001, -5, 70_000, 12),
             ("uniform", 1_500_000, 7, 7 + (1 << 18), 13), ("uniform", 3_000_000, 0, 1 << 22, 14)]
    cases = []
    for dist, n, lo, hi, seed in specs:
        A = inputs.make(dist, n, lo, hi, seed)
        _, t = _to_dev(A)
        cases.append((t, lo, hi, oracle.sort(A, lo, hi)))
    torch.cuda.synchronize()
    errors = []

    def work(k):
        try:
            s = torch.cuda.Stream()
            order = [(k + j) % len(cases) for j in range(len(cases))]
            for _ in range(3):
                outs = []
                with torch.cuda.stream(s):
                    for i in order:
                        t, lo, hi, _ = cases[i]
                        outs.append((i, r.sort(t, lo, hi)))
                s.synchronize()
                for i, o in outs:
                    if not np.array_equal(o.cpu().numpy(), cases[i][3]):
                        errors.append((k, i))
        except Exception as e:   # reported by the main thread
            errors.append((k, repr(e)))

    _say("four host threads, one stream each")
    threads = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors


def test_host_threads_one_stream(r):
    """Three host threads sorting on one stream (the current stream of each,
    the device's default one), so that their sorts share one cached workspace
    and fast-path area: problems of growing workspace size in different
    orders, so the workspace grows (after a wait for that stream) while
    another thread's sorts are queued on it.  Every output equals the
    oracle's."""
    import threading
    r.release_workspaces()
    specs = [("uniform", 300_001, 0, 1000, 21), ("normal", 1_000_003, -9, 1 << 16, 22),
             ("uniform", 2_000_000, 5, 5 + (1 << 18), 23), ("uniform", 4_000_000, 0, 1 << 22, 24)]
    cases = []
    for dist, n, lo, hi, seed in specs:
        A = inputs.make(dist, n, lo, hi, seed)
        _, t = _to_dev(A)
        cases.append((t, lo, hi, oracle.sort(A, lo, hi)))
    torch.cuda.synchronize()
    errors = []

    def work(k):
        try:
            order = list(range(len(cases))) if k == 0 else [(k + j) % len(cases) for j in range(len(cases))][::-1]
            outs = [(i, r.sort(cases[i][0], cases[i][1], cases[i][2])) for _ in range(2) for i in order]
            torch.cuda.current_stream().synchronize()
            for i, o in outs:
                if not np.array_equal(o.cpu().numpy(), cases[i][3]):
                    errors.append((k, i))
        except Exception as e:   # reported by the main thread
            errors.append((k, repr(e)))

    _say("three host threads, one stream")
    threads = [threading.Thread(target=work, args=(k,)) for k in range(3)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors


def test_empty_and_errors(r):
    t = torch.empty(0, dtype=torch.int32, device="cuda")
    assert r.sort(t, 0, 10).numel() == 0
    x = torch.zeros(100, dtype=torch.int32, device="cuda")
    assert r.lib.rtcdf_sort(r._ptr(x), r._ptr(x[10:]), 50, 0, 10, None) == r.OVERLAP
    with pytest.raises(r.RtcdfError) as e:
        r.sort(x, 0, 10, config=r.make_config(32768, 16, 2))
    assert e.value.status == r.INVALID_VALUE


def test_fast_path_plan(r):
    """One tile, one pass of 32-bit counters, R <= 2048 and fewer than 2^26
    int32 keys (2^28 bytes) take the fast path (histogram and output stage only: no local-CDF workgroups);
    other plans keep every stage."""
    for n in (10_000_000, (1 << 26) - 1, 1 << 26, 100_000_000):
        for R in (1, 128, 1000, 2048, 2049, 5000, 1 << 16):
            info = r.plan_info(n, 0, R)
            _say(f"plan n={n} R={R} {info}")
            fast = (info["tiles"] == 1 and info["counter_bits"] == 32 and info["passes"] == 1 and R <= 2048
                    and n < (1 << 26))
            assert (info["scan_workgroups"] == 0) == fast
            if R <= 128:
                assert fast == (n < (1 << 26))


def test_fast_path_sequence(r):
    """Fast, staged and narrow-counter sorts interleaved on one stream: the
    fast path's accumulation area must be left consistent by every sort."""
    rng = np.random.default_rng(31)
    s = torch.cuda.Stream()
    cases = [
        (1_000_000, 128, "uniform", None),
        (300_000, 2048, "normal", None),
        (500_000, 70_000, "uniform", None),        # 8-bit counters, staged
        (1000, 1, "uniform", None),
        (10, 2000, "uniform", None),               # fewer keys than values
        (2_000_001, 300, "zipf", None),
        (400_000, 2048, "uniform", r.make_config(1024, 16, 1)),   # two tiles: staged
        (1_000_000, 128, "all_equal", None),
        (77_777, 1500, "normal", None),
    ]
    for rep in range(2):
        for i, (n, R, dist, cfg) in enumerate(cases):
            lo = int(rng.integers(-5000, 5000))
            A = inputs.make(dist, n, lo, lo + R, 1000 * rep + i)
            want = oracle.sort(A, lo, lo + R)
            _, tin = _to_dev(A, i % 4)
            _say(f"sequence rep={rep} n={n} R={R} {dist} cfg={cfg}")
            with torch.cuda.stream(s):
                out = r.sort(tin, lo, lo + R, config=cfg, stream=s)
            s.synchronize()
            assert np.array_equal(out.cpu().numpy(), want)


def test_fast_path_graph_replay(r):
    """Captured fast-path sorts (library workspace and caller workspace)
    replay correctly with new inputs between replays: the fast path keeps its
    state on the device."""
    n, R = 300_001, 1000
    s = torch.cuda.Stream()
    tin = torch.empty(n, dtype=torch.int32, device="cuda")
    out1 = torch.empty_like(tin)
    out2 = torch.empty_like(tin)
    ws = torch.empty(r.workspace_bytes(n, 0, R, keys_out=out2), dtype=torch.uint8, device="cuda")
    ws.fill_(0xCD)
    tin.copy_(torch.from_numpy(inputs.uniform(n, 0, R, 5)))
    _say("fast path graph: warm-up")
    with torch.cuda.stream(s):
        r.sort(tin, 0, R, keys_out=out1, stream=s)    # allocates the library workspace
        r.sort_ws(tin, out2, 0, R, ws, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        r.sort(tin, 0, R, keys_out=out1, stream=s)
        r.sort_ws(tin, out2, 0, R, ws, stream=s)
    for rep in range(4):
        dist = ("uniform", "normal", "zipf", "all_equal")[rep]
        A = inputs.make(dist, n, 0, R, 50 + rep)
        want = oracle.sort(A, 0, R)
        tin.copy_(torch.from_numpy(A))
        out1.fill_(-1)
        out2.fill_(-1)
        torch.cuda.synchronize()
        _say(f"fast path graph: replay {rep} {dist}")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out1.cpu().numpy(), want)
        assert np.array_equal(out2.cpu().numpy(), want)
        # an eager sort on the same stream between replays
        with torch.cuda.stream(s):
            r.sort(tin, 0, R, keys_out=out1, stream=s)
        s.synchronize()
        assert np.array_equal(out1.cpu().numpy(), want)
    # Releasing the library's workspaces keeps the ones a capture used: the
    # graph still replays correctly afterwards, and a larger sort on the same
    # stream (which grows the workspace) retires the captured buffers instead
    # of freeing them.
    r.release_workspaces()
    big = torch.from_numpy(inputs.uniform(3_000_000, 0, 1 << 16, 58)).cuda()
    with torch.cuda.stream(s):
        r.sort(big, 0, 1 << 16, stream=s)
    s.synchronize()
    A = inputs.make("normal", n, 0, R, 59)
    tin.copy_(torch.from_numpy(A))
    out1.fill_(-1)
    torch.cuda.synchronize()
    _say("fast path graph: replay after release and growth")
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(out1.cpu().numpy(), oracle.sort(A, 0, R))


def test_capture_without_workspace_is_refused(r):
    """rtcdf_sort on a stream whose library workspace does not exist yet
    cannot allocate under capture: it returns CAPTURE_NEEDS_WORKSPACE and
    enqueues nothing."""
    n, R = 100_000, 5000
    tin = torch.from_numpy(inputs.uniform(n, 0, R, 60)).cuda()
    out = torch.empty_like(tin)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    _say("capture without a workspace")
    with pytest.raises(r.RtcdfError) as ei:
        with torch.cuda.graph(g, stream=s):
            r.sort(tin, 0, R, keys_out=out, stream=s)
    assert ei.value.status == r.CAPTURE_NEEDS_WORKSPACE
    # the stream works normally afterwards
    with torch.cuda.stream(s):
        r.sort(tin, 0, R, keys_out=out, stream=s)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.sort(tin.cpu().numpy(), 0, R))


@pytest.mark.parametrize("n", [65536 * 1 + 4, 65536 * 2 + 1, 65536 * 3 + 3, 65536 * 8 + 2, 262_147])
def test_caller_workspace_alignments(r, n):
    """rtcdf_workspace_bytes is asked with keys_out only; the workspace it
    reports suffices whatever the alignment of keys_in (the histogram's
    workgroup count does not depend on it), including n where the input body
    crosses a multiple of the histogram's keys per workgroup round."""
    R = 1000
    A = inputs.uniform(n, -3, -3 + R, n)
    want = oracle.sort(A, -3, -3 + R)
    for oi in range(4):
        for oo in range(4):
            if oi == oo:
                continue
            bi = torch.empty(n + 4, dtype=torch.int32, device="cuda")
            bo = torch.empty(n + 4, dtype=torch.int32, device="cuda")
            tin, out = bi[oi:oi + n], bo[oo:oo + n]
            tin.copy_(torch.from_numpy(A))
            nb = r.workspace_bytes(n, -3, -3 + R, keys_out=out)
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
            _say(f"sort_ws alignment n={n} in+{oi} out+{oo} bytes={nb}")
            r.sort_ws(tin, out, -3, -3 + R, ws)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), want)


def test_checked_mode(r):
    """Checked mode counts the keys outside [minVal, maxVal) (in the scalar head,
    the vector body and the tail of unaligned arrays; on both sides of the
    range; int32 extremes) and refuses to sort them, leaving the output
    untouched, as the oracle refuses them; in-range keys sort as usual."""
    rng = np.random.default_rng(77)
    I32 = np.iinfo(np.int32)
    lo, R = -50, 300
    for n, pin in ((1, 0), (3, 1), (7, 2), (1000, 3), (1_000_003, 1)):
        A = rng.integers(lo, lo + R, size=n).astype(np.int32)
        _, tin = _to_dev(A, pin)
        _say(f"checked n={n} pin={pin} in range")
        c = r.count_out_of_range(tin, lo, lo + R)
        torch.cuda.synchronize()
        assert int(c.item()) == 0
        out = r.sort_checked(tin, lo, lo + R)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.sort(A, lo, lo + R))
        # keys planted at the first and last position and a few in between
        B = A.copy()
        idx = sorted(set([0, n - 1] + [int(i) for i in rng.integers(0, n, size=min(n, 5))]))
        vals = [lo - 1, lo + R, I32.min, I32.max, lo - 1000]
        for j, i in enumerate(idx):
            B[i] = vals[j % len(vals)]
        wide = B.astype(np.int64)
        want_bad = int(np.count_nonzero((wide < lo) | (wide >= lo + R)))
        with pytest.raises(oracle.OracleError) as e:
            oracle.sort(B, lo, lo + R)
        assert e.value.code == oracle.ORC_KEY_OUT_OF_RANGE
        _, tb = _to_dev(B, pin)
        _say(f"checked n={n} pin={pin} out of range: {want_bad}")
        c = r.count_out_of_range(tb, lo, lo + R)
        torch.cuda.synchronize()
        assert int(c.item()) == want_bad
        out = torch.full_like(tb, 0x5A5A5A5A)
        with pytest.raises(r.RtcdfError) as e:
            r.sort_checked(tb, lo, lo + R, keys_out=out)
        assert e.value.status == r.KEY_OUT_OF_RANGE
        torch.cuda.synchronize()
        assert np.all(out.cpu().numpy() == 0x5A5A5A5A)


def test_release_workspaces_between_sorts(r):
    """Released library workspaces (plain, carry and fast-path areas) are
    re-created zeroed: sorts before and after a release agree with the oracle."""
    rng = np.random.default_rng(123)
    for rep in range(2):
        for R in (100, 2000, 70000):
            A = rng.integers(0, R, size=200_003).astype(np.int32)
            _, tin = _to_dev(A, rep)
            _say(f"release rep={rep} R={R}")
            out = r.sort(tin, 0, R)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), oracle.sort(A, 0, R))
        assert r.lib.rtcdf_release_workspaces() == r.SUCCESS
