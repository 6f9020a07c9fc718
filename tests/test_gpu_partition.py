"""GPU parity of the partition by LDS pass (wide ranges) against the CPU oracle:
forced on at small sizes (ragged n, every distribution, misaligned and in-place
outputs, the Alg. 4-6 intermediates, caller workspace and graph replays),
forced off as the reference, and the library's own choice at full size."""
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


@pytest.fixture
def forced(monkeypatch):
    monkeypatch.setenv("RTCDF_DEV_PARTITION", "1")


def _check(r, A, minVal, maxVal, cfg=None, pin=0, pout=0, inplace=False):
    _say(f"part n={A.size} min={minVal} R={maxVal - minVal} cfg={cfg} pin={pin} pout={pout} inplace={inplace}")
    want = oracle.sort(A, minVal, maxVal)
    bin_ = torch.full((A.size + pin + 4,), -7, dtype=torch.int32, device="cuda")
    tin = bin_[pin:pin + A.size]
    tin.copy_(torch.from_numpy(np.ascontiguousarray(A, dtype=np.int32)))
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
    assert np.array_equal(tin.cpu().numpy(), np.asarray(A, dtype=np.int32))


def test_plan(r, monkeypatch):
    """The library partitions from 9 passes on when n x passes >= 2^26; the
    override forces it wherever there are at least 2 passes."""
    p = lambda n, R: r.plan_info(n, 0, R)
    assert p(10 ** 8, 1 << 22)["partition_buckets"] == p(10 ** 8, 1 << 22)["passes"] > 8
    assert p(10 ** 8, 1 << 20)["partition_buckets"] == 0          # 7 passes
    assert p(10 ** 8, 1 << 18)["partition_buckets"] == 0          # two passes
    assert p(10 ** 6, 1 << 22)["partition_buckets"] == 0          # 26 passes, n x passes < 2^26
    assert p(4 * 10 ** 6, 1 << 22)["partition_buckets"] > 0
    assert p(10 ** 6, 1 << 24)["partition_buckets"] > 0
    assert p(10 ** 8, 1 << 16)["partition_buckets"] == 0          # one pass
    monkeypatch.setenv("RTCDF_DEV_PARTITION", "1")
    assert p(1000, 1 << 18)["partition_buckets"] == 2
    assert p(1000, 1 << 16)["partition_buckets"] == 0
    monkeypatch.setenv("RTCDF_DEV_PARTITION", "0")
    assert p(10 ** 8, 1 << 22)["partition_buckets"] == 0


@pytest.mark.parametrize("R", [1 << 18, (1 << 20) + 3, 1 << 22])
def test_ragged_sizes(r, forced, R):
    rng = np.random.default_rng(R)
    for i, n in enumerate((1, 2, 3, 5, 4095, 4096, 4097, 65537, 300001)):
        minVal = int(rng.integers(-10 ** 6, 10 ** 6))
        A = rng.integers(minVal, minVal + R, size=n).astype(np.int32)
        _check(r, A, minVal, minVal + R, pin=i % 4, pout=(i + 1) % 4)


@pytest.mark.parametrize("dist", ["uniform", "normal", "all_equal", "zipf"])
@pytest.mark.parametrize("R", [1 << 19, 1 << 22, 1 << 24])
def test_distributions(r, forced, dist, R):
    A = inputs.make(dist, 2_000_003, -1000, -1000 + R, inputs.case_seed(11, R % 97))
    _check(r, A, -1000, -1000 + R, pout=2)


def test_in_place_extremes_and_grid(r, forced):
    rng = np.random.default_rng(4)
    A = rng.integers(0, 1 << 21, size=500_001).astype(np.int32)
    _check(r, A, 0, 1 << 21, inplace=True)
    lo = -2 ** 31
    A = rng.integers(lo, lo + (1 << 20), size=200_000, dtype=np.int64).astype(np.int32)
    _check(r, A, lo, lo + (1 << 20))
    hi = 2 ** 31
    A = rng.integers(hi - (1 << 20), hi, size=200_000, dtype=np.int64).astype(np.int32)
    _check(r, A, hi - (1 << 20), hi)
    A = inputs.make("normal", 300_001, 0, 1 << 20, 5)
    for T, items, bpt in ((1024, 4, 1), (8192, 16, 2), (32768, 8, 1), (4096, 16, 4)):
        _check(r, A, 0, 1 << 20, r.make_config(T, items, bpt))
    # with the prefix-maximum output too
    _check(r, A, 0, 1 << 20, r.make_config(4096, 16, 1, flags=r.FLAG_OUTPUT_PREFIX_MAX))


@pytest.mark.parametrize("R,T", [(300000, 8192), ((1 << 20) + 5, 32768)])
def test_intermediates(r, forced, R, T):
    rng = np.random.default_rng(R)
    A = rng.integers(-9, -9 + R, size=250_001).astype(np.int32)
    A[:777] = -9 + R - 1
    Teff = min(T, (R + 127) // 128 * 128)
    _say(f"part intermediates R={R} T={T}")
    h, c, O = oracle.tile_intermediates(A, -9, -9 + R, Teff)
    tin = torch.from_numpy(A).cuda()
    gh, gc, gO = r.debug_intermediates(tin, -9, -9 + R, r.make_config(T, 16, 1))
    torch.cuda.synchronize()
    as_u = lambda t: t.cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal(as_u(gh), h)
    assert np.array_equal(as_u(gc), c)
    assert np.array_equal(as_u(gO), O)


def test_caller_workspace_graph_replay(r, forced):
    n, R = 300_001, 1 << 21
    s = torch.cuda.Stream()
    tin = torch.empty(n, dtype=torch.int32, device="cuda")
    out = torch.empty_like(tin)
    ws = torch.empty(r.workspace_bytes(n, 0, R, keys_out=out), dtype=torch.uint8, device="cuda")
    ws.fill_(0xCD)
    tin.copy_(torch.from_numpy(inputs.uniform(n, 0, R, 3)))
    _say("part graph: warm-up")
    with torch.cuda.stream(s):
        r.sort_ws(tin, out, 0, R, ws, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        r.sort_ws(tin, out, 0, R, ws, stream=s)
    for rep, dist in enumerate(("uniform", "normal", "zipf", "all_equal")):
        A = inputs.make(dist, n, 0, R, 70 + rep)
        want = oracle.sort(A, 0, R)
        tin.copy_(torch.from_numpy(A))
        out.fill_(-1)
        ws.fill_(0xCD)
        torch.cuda.synchronize()
        _say(f"part graph: replay {rep} {dist}")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want)
        with torch.cuda.stream(s):
            r.sort_ws(tin, out, 0, R, ws, stream=s)
        s.synchronize()
        assert np.array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("dist", ["uniform", "normal", "zipf", "all_equal"])
def test_library_choice_full_size(r, dist):
    """n = 10^8, R = 2^22 (26 passes): the library partitions; every key is
    checked against the oracle's counts by the streaming verifier.  Zipf and
    all-equal keys put nearly every key in one bucket, whose pieces then span
    most of the histogram workgroups."""
    n, R = 10 ** 8, 1 << 22
    assert r.plan_info(n, 0, R)["partition_buckets"] > 0
    a = inputs.make_device(dist, n, 0, R, 13)
    b = torch.empty_like(a)
    _say(f"part full size {dist}")
    r.sort(a, 0, R, keys_out=b)
    torch.cuda.synchronize()
    cnt = np.zeros(R, dtype=np.uint64)
    for i in range(0, n, 1 << 26):
        cnt += oracle.counts(a[i:i + (1 << 26)].cpu().numpy(), 0, R)
    v = oracle.StreamingVerifier(cnt, 0)
    for i in range(0, n, 1 << 26):
        v.chunk(b[i:i + (1 << 26)].cpu().numpy())
    v.end(n)
