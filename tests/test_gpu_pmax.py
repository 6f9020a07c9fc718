"""GPU parity of the prefix-maximum output method (Alg. 3, selected with
RTCDF_FLAG_OUTPUT_PREFIX_MAX) against the CPU oracle, element by element:
ragged sizes around its 8192-position chunks and 1024-position windows,
misaligned and in-place outputs, every valid grid point, the caller-workspace
form and graph replays."""
import sys

import numpy as np
import pytest

import oracle
from paper_2609_00843_amd import inputs

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


def _cfg(r, T=4096, items=16, bpt=1):
    return r.make_config(T, items, bpt, flags=r.FLAG_OUTPUT_PREFIX_MAX)


def _check(r, A, minVal, maxVal, cfg, pout=0, inplace=False):
    _say(f"pmax n={A.size} min={minVal} max={maxVal} cfg={cfg} pout={pout} inplace={inplace}")
    want = oracle.sort(A, minVal, maxVal)
    tin = torch.from_numpy(np.ascontiguousarray(A, dtype=np.int32)).cuda()
    if inplace:
        r.sort(tin, minVal, maxVal, keys_out=tin, config=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(tin.cpu().numpy(), want)
        return
    buf = torch.full((A.size + pout + 8,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    out = buf[pout:pout + A.size]
    r.sort(tin, minVal, maxVal, keys_out=out, config=cfg)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got, want), f"mismatch at {np.flatnonzero(got != want)[:8]}"
    full = buf.cpu().numpy()
    assert np.all(full[:pout] == 0x5A5A5A5A) and np.all(full[pout + A.size:] == 0x5A5A5A5A)


@pytest.mark.parametrize("R", [1, 2, 129, 4097, 65537, 262144])
def test_ragged_sizes(r, R):
    rng = np.random.default_rng(R + 1)
    for i, n in enumerate((1, 2, 3, 4, 5, 1023, 1024, 1025, 8191, 8192, 8193, 8195, 16387, 300001)):
        minVal = int(rng.integers(-10 ** 6, 10 ** 6))
        A = rng.integers(minVal, minVal + R, size=n).astype(np.int32)
        _check(r, A, minVal, minVal + R, _cfg(r, 1024 if R < 4097 else 8192), pout=i % 4)


@pytest.mark.parametrize("dist", ["uniform", "normal", "all_equal", "zipf"])
@pytest.mark.parametrize("logR", [7, 13, 16, 18])
def test_distributions(r, dist, logR):
    R = 1 << logR
    A = inputs.make(dist, 2_000_003, -1000, -1000 + R, inputs.case_seed(9, logR))
    _check(r, A, -1000, -1000 + R, _cfg(r, min(R, 8192)), pout=logR % 4)


@pytest.mark.parametrize("n,pout", [((1 << 21) - 1, 0), (1 << 21, 3), ((1 << 21) + 1, 1), (3_000_001, 2),
                                    (8192 * 1024 - 3, 1), (8192 * 1024 + 5, 0)])
def test_chunk_regimes(r, n, pout):
    """Around the switch from 2048- to 8192-position chunks (n = 2^21) and from
    carries computed by each wave to the carry kernel (more than 1024 chunks)."""
    R = 1 << 16
    A = inputs.make("normal", n, 5, 5 + R, n % 1000)
    _check(r, A, 5, 5 + R, _cfg(r, 8192), pout=pout)


def test_in_place_and_extremes(r):
    rng = np.random.default_rng(3)
    A = rng.integers(0, 70000, size=500_001).astype(np.int32)
    _check(r, A, 0, 70000, _cfg(r), inplace=True)
    lo, hi = 2 ** 31 - 1000, 2 ** 31
    A = rng.integers(lo, hi, size=100_000, dtype=np.int64).astype(np.int32)
    _check(r, A, lo, hi, _cfg(r, 1024))
    lo = -2 ** 31
    A = rng.integers(lo, lo + 300, size=100_000, dtype=np.int64).astype(np.int32)
    _check(r, A, lo, lo + 300, _cfg(r, 128, 4, 4))


def test_every_grid_point(r):
    cfgs, valid = r.config_grid()
    A = inputs.make("normal", 400_001, 7, 7 + 20000, 11)
    want = oracle.sort(A, 7, 7 + 20000)
    tin = torch.from_numpy(A).cuda()
    out = torch.empty_like(tin)
    for (T, items, bpt, flags), ok in zip(cfgs, valid):
        if not ok or flags:     # the plain points (the option points carry their own flags)
            continue
        _say(f"pmax grid T={T} items={items} bpt={bpt}")
        out.fill_(-1)
        r.sort(tin, 7, 7 + 20000, keys_out=out, config=_cfg(r, T, items, bpt))
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want)


def test_caller_workspace_graph_replay(r):
    """sort_ws with the prefix-maximum output, eager and captured; every replay
    (new inputs between replays, an eager sort on the same stream after each)
    matches the oracle."""
    n, R = 300_001, 70000
    cfg = _cfg(r, 8192)
    s = torch.cuda.Stream()
    tin = torch.empty(n, dtype=torch.int32, device="cuda")
    out = torch.empty_like(tin)
    ws = torch.empty(r.workspace_bytes(n, 0, R, config=cfg, keys_out=out), dtype=torch.uint8,
                     device="cuda")
    ws.fill_(0xCD)
    tin.copy_(torch.from_numpy(inputs.uniform(n, 0, R, 5)))
    _say("pmax graph: warm-up")
    with torch.cuda.stream(s):
        r.sort_ws(tin, out, 0, R, ws, config=cfg, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        r.sort_ws(tin, out, 0, R, ws, config=cfg, stream=s)
    for rep, dist in enumerate(("uniform", "normal", "zipf", "all_equal")):
        A = inputs.make(dist, n, 0, R, 60 + rep)
        want = oracle.sort(A, 0, R)
        tin.copy_(torch.from_numpy(A))
        out.fill_(-1)
        ws.fill_(0xCD)
        torch.cuda.synchronize()
        _say(f"pmax graph: replay {rep} {dist}")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want)
        with torch.cuda.stream(s):
            r.sort_ws(tin, out, 0, R, ws, config=cfg, stream=s)
        s.synchronize()
        assert np.array_equal(out.cpu().numpy(), want)


def test_same_output_as_interval_fill(r):
    """The two output methods agree byte for byte on the same input and tile
    width, including n = 10^7 with a ragged tail."""
    A = inputs.make("normal", 10_000_003, 0, 1 << 16, 77)
    tin = torch.from_numpy(A).cuda()
    a = torch.empty_like(tin)
    b = torch.empty_like(tin)
    _say("pmax vs interval fill n=10^7+3 R=2^16")
    r.sort(tin, 0, 1 << 16, keys_out=a, config=r.make_config(8192, 16, 1))
    r.sort(tin, 0, 1 << 16, keys_out=b, config=_cfg(r, 8192))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert np.array_equal(b.cpu().numpy(), oracle.sort(A, 0, 1 << 16))


def test_library_choice_rule(r):
    """The library's own choice writes the output by the prefix maximum exactly
    when R >= 2^14 and R >= n, in plan_info and pick_config alike; an explicit
    config keeps its own output method."""
    for n, R in ((1000, 1 << 14), (1000, (1 << 14) - 1), (16384, 1 << 14), (16385, 1 << 14),
                 (10 ** 5, 1 << 18), (10 ** 6, 1 << 18), (10 ** 6, 1 << 22), (10 ** 8, 1 << 18),
                 (5, 2048), (3000, 1 << 28)):
        want = r.FLAG_OUTPUT_PREFIX_MAX if (R >= 1 << 14 and R >= n) else 0
        info = r.plan_info(n, 0, R)
        _say(f"rule n={n} R={R} -> {info['output_flags']}")
        assert info["output_flags"] == want
        assert r.pick_config(n, 0, R).flags == want
        assert r.plan_info(n, 0, R, config=r.make_config(4096))["output_flags"] == 0
        assert r.plan_info(n, 0, R, config=_cfg(r))["output_flags"] == r.FLAG_OUTPUT_PREFIX_MAX


@pytest.mark.parametrize("dist", ["uniform", "normal", "all_equal", "zipf"])
def test_library_choice_parity(r, dist):
    """Sorts with the library's choice on both sides of the rule."""
    for n, logR in ((3000, 18), (100_000, 20), (100_000, 16), (20_000, 14)):
        R = 1 << logR
        A = inputs.make(dist, n, -5000, -5000 + R, n + logR)
        _check(r, A, -5000, -5000 + R, None, pout=n % 4)
