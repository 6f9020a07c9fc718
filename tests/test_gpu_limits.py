"""GPU parity at the limits the boundary accepts: n up to 2^32 - 1 keys (the
largest count a 32-bit counter holds, reading iv of the counter width) and
ranges up to RTCDF_MAX_RANGE = 2^28.

Near n = 2^32 the output positions of the last steps lie within a step of
2^32, where an end position p + 256 no longer fits 32 bits.  The inputs
therefore plant rare values at the top of the range, so that several value
boundaries (and, for the sparse form, a window of many values) fall inside
the last output step.  Every output element is compared with the oracle's
counts by the streaming verifier; the counts come from chunked copies of the
input."""
import sys

import numpy as np
import pytest

import oracle
from paper_2609_00843_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CHUNK = 1 << 26
N32 = (1 << 32) - 1


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def r():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_00843_amd import rtcdf
    return rtcdf


def _planted(n, lo, hi, gap, tail, seed, dtype=torch.int32, skip=0):
    """n keys: uniform over [lo + skip, hi - gap) except the last keys of the
    array, which are `tail` = [(value, copies), ...] (values outside the
    uniform body's range, so their counts are exactly as planted)."""
    k = sum(c for _, c in tail)
    a = torch.empty(n, dtype=dtype, device="cuda")
    body = inputs.make_device("uniform", n - k, lo + skip, hi - gap, seed)
    a[:n - k] = body.to(dtype)
    del body
    vals = np.concatenate([np.full(c, v, dtype=np.int64) for v, c in tail])
    a[n - k:] = torch.from_numpy(vals).to(dtype).cuda()
    return a


def _counts(a, lo, hi):
    R = hi - lo
    cnt = np.zeros(R, dtype=np.uint64)
    for s in range(0, a.numel(), CHUNK):
        cnt += oracle.counts(a[s:s + CHUNK].cpu().numpy().astype(np.int32), lo, hi)
    return cnt


def _verify(b, cnt, lo, n):
    v = oracle.StreamingVerifier(cnt, lo)
    for s in range(0, n, CHUNK):
        v.chunk(b[s:s + CHUNK].cpu().numpy().astype(np.int32))
    v.end(n)


@pytest.mark.parametrize("n,lo,R,skip,gap,tail", [
    # one tile of 128 values (the staged path: the single-tile fast path
    # stops at 2^28 bytes of keys), dense output walk over the last step
    (N32, -1000, 1 << 7, 0, 8, [(-1000 + 120, 3), (-1000 + 122, 1), (-1000 + 123, 60), (-1000 + 127, 100)]),
    # staged path, 8-bit counters.  200 rare values at the bottom make the
    # first output chunk's window sparse, which switches the output stage to
    # its per-chunk choice; the last chunk's window then holds ~200 values over
    # ~100 positions and takes the sparse form (scatter over LDS)
    (N32, 5, 1 << 16, 400, 200, [(5 + 2 * j, 1) for j in range(200)] +
     [(5 + (1 << 16) - 200 + 2 * j, 1) for j in range(100)]),
    # above 2^31: two passes of 8-bit counters
    ((1 << 31) + (1 << 20), 0, 1 << 18, 0, 16, [((1 << 18) - 16, 7), ((1 << 18) - 3, 250), ((1 << 18) - 1, 9)]),
])
def test_int32_near_2pow32(r, n, lo, R, skip, gap, tail):
    hi = lo + R
    _say(f"int32 n={n} R={R} planted tail of {sum(c for _, c in tail)} keys, output at 4 mod 16 bytes")
    a = _planted(n, lo, hi, gap, tail, inputs.case_seed(60, R), skip=skip)
    cnt = _counts(a, lo, hi)
    assert int(cnt.sum()) == n
    buf = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    b = buf[1:]                       # 4-byte offset: a scalar head and an unaligned body end
    r.sort(a, lo, hi, keys_out=b)
    torch.cuda.synchronize()
    del a
    _verify(b, cnt, lo, n)


def test_uint8_near_2pow32(r):
    """n = 2^32 - 1 uint8 keys over the whole type (the dense output form
    writes 16 keys per lane and step, 1024 positions per wave)."""
    n, lo, hi = N32, 0, 256
    tail = [(248, 5), (250, 1), (251, 300), (255, 40)]
    _say(f"uint8 n={n} planted tail")
    a = _planted(n, lo, hi, 8, tail, inputs.case_seed(61, 0), dtype=torch.uint8)
    cnt = _counts(a, lo, hi)
    b = torch.empty_like(a)
    r.sort_keys(a, lo, hi, keys_out=b)
    torch.cuda.synchronize()
    del a
    _verify(b, cnt, lo, n)


def test_batched_segment_near_2pow32(r):
    """One batch segment of 2^32 - 1 keys (two range tiles, each one
    workgroup's item end to end: segments are not split over workgroups)
    beside a small one; the error word of timed-out waits stays zero."""
    n, lo, R = N32, -77, 40000
    tail = [(lo + R - 30, 2), (lo + R - 29, 1), (lo + R - 1, 80)]
    _say(f"batched segment n={n} R={R}")
    a = _planted(n, lo, lo + R, 30, tail, inputs.case_seed(62, 0))
    cnt = _counts(a, lo, lo + R)
    b = torch.empty_like(a)
    small = torch.from_numpy(inputs.uniform(1001, 3, 103, 9)).cuda()
    small_out = torch.empty_like(small)
    d, bounds, k = r.make_segments([(a, b, lo, lo + R), (small, small_out, 3, 103)])
    ws = torch.empty(r.batched_workspace_bytes(k, bounds), dtype=torch.uint8, device="cuda")
    r.sort_batched(d, k, bounds, ws)
    torch.cuda.synchronize()
    del a
    assert int(ws[8:12].cpu().view(torch.int32).item()) == 0   # no timed-out wait
    assert np.array_equal(small_out.cpu().numpy(), oracle.sort(small.cpu().numpy(), 3, 103))
    _verify(b, cnt, lo, n)


@pytest.mark.parametrize("n,lo,logR,dist,search", [
    (10_000_003, -(1 << 27), 26, "uniform", False),
    (10_000_003, -(1 << 27), 26, "normal", True),
    (10_000_001, (1 << 31) - (1 << 28), 28, "uniform", False),   # maxVal = 2^31
    (10_000_001, -(1 << 31), 28, "normal", True),                # minVal = INT32_MIN
])
def test_widest_ranges(r, n, lo, logR, dist, search):
    """R = 2^26 and 2^28 (the largest accepted range), n = 10^7: the library's
    choice (the prefix-maximum output, since R > n) and the search output with
    an explicit configuration (its sparse form); both partition the keys by
    pass."""
    R = 1 << logR
    hi = lo + R
    A = inputs.make(dist, n, lo, hi, inputs.case_seed(63, logR))
    cfg = r.make_config(8192, 8, 1) if search else None
    info = r.plan_info(n, lo, hi, config=cfg)
    _say(f"R=2^{logR} {dist} n={n} lo={lo} search={search} plan={info}")
    a = torch.from_numpy(A).cuda()
    b = torch.empty(n + 3, dtype=torch.int32, device="cuda")[3:]
    r.sort(a, lo, hi, keys_out=b, config=cfg)
    torch.cuda.synchronize()
    assert info["partition_buckets"] > 0
    assert info["output_flags"] == (0 if search else r.FLAG_OUTPUT_PREFIX_MAX)
    assert np.array_equal(b.cpu().numpy(), oracle.sort(A, lo, hi))
