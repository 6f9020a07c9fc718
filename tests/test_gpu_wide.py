"""GPU parity of sorts of n >= 2^32 keys, whose per-value counts and output
positions need 64 bits (rtcdf_wide.hip: the input counted in pieces of 2^31
keys into 64-bit counts, the output written in windows of 2^31 positions).

The oracle side is the counting sort's definition with 64-bit counts (Sec.
2.1): the counts c_v of the input, summed over chunks in uint64, and the
streaming verifier, which expands them in value order against the output
chunk by chunk (its 64-bit cursor is pinned on the CPU in test_oracle).  The
cases cross piece and window boundaries inside a value's run of copies, hold
one value more than 2^32 times, take the caller-workspace form in place with
the keys partitioned by pass, and sort int64 and uint8 keys."""
import sys

import numpy as np
import pytest

import oracle
from paper_2609_00843_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CHUNK = 1 << 26
PIECE = 1 << 31


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def r():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_00843_amd import rtcdf
    return rtcdf


def _norm(chunk, lo):
    """Values of a device chunk as offsets from lo, int32 on the host."""
    return (chunk.to(torch.int64) - lo).to(torch.int32).cpu().numpy()


def _counts(a, lo, R):
    cnt = np.zeros(R, dtype=np.uint64)
    for s in range(0, a.numel(), CHUNK):
        cnt += oracle.counts(_norm(a[s:s + CHUNK], lo), 0, R)
    return cnt


def _verify(b, cnt, lo, n):
    v = oracle.StreamingVerifier(cnt, 0)
    for s in range(0, n, CHUNK):
        v.chunk(_norm(b[s:s + CHUNK], lo))
    v.end(n)


def _uniform(n, lo, hi, seed, dtype):
    """n keys uniform over [lo, hi), generated in chunks on the GPU."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    a = torch.empty(n, dtype=dtype, device="cuda")
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        a[s:e] = (torch.randint(0, hi - lo, (e - s,), generator=g, device="cuda", dtype=torch.int64) + lo).to(dtype)
    return a


def _plant(a, tail):
    """The last keys of a become `tail` = [(value, copies), ...]."""
    vals = np.concatenate([np.full(c, v, dtype=np.int64) for v, c in tail])
    a[a.numel() - vals.size:] = torch.from_numpy(vals).to(a.dtype).cuda()


def test_int32_wide(r):
    """Three pieces (2^31, 2^31, 2^21 + 5 keys) over R = 2^16 with 8-bit
    counters; values planted at the top of the range so that the last window
    ends in a few rare values; the output at 4 mod 16 bytes."""
    n, lo, R = 2 * PIECE + (1 << 21) + 5, -1000, 1 << 16
    _say(f"int32 n={n} R={R} (three pieces and windows), output at 4 mod 16 bytes")
    a = _uniform(n, lo, lo + R - 32, inputs.case_seed(70, R), torch.int32)
    _plant(a, [(lo + R - 20, 3), (lo + R - 7, 1000), (lo + R - 1, 77)])
    cnt = _counts(a, lo, R)
    assert int(cnt.sum()) == n
    buf = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    b = buf[1:]
    r.sort(a, lo, lo + R, keys_out=b)
    torch.cuda.synchronize()
    del a
    _verify(b, cnt, lo, n)


def test_uint8_value_over_2pow32(r):
    """One value held more than 2^32 times (its 64-bit count spans all three
    output windows), beside 2^22 uniform keys and a planted tail."""
    n, lo, hi = 2 * PIECE + (1 << 22) + 3, 0, 256
    _say(f"uint8 n={n}, value 200 more than 2^32 times")
    a = torch.full((n,), 200, dtype=torch.uint8, device="cuda")
    a[:1 << 22] = _uniform(1 << 22, lo, hi, inputs.case_seed(71, 0), torch.uint8)
    _plant(a, [(0, 5), (255, 9)])
    cnt = _counts(a, lo, hi - lo)
    assert int(cnt[200]) > (1 << 32)
    b = torch.empty_like(a)
    r.sort_keys(a, lo, hi, keys_out=b)
    torch.cuda.synchronize()
    del a
    _verify(b, cnt, lo, n)


def test_int64_wide(r):
    """int64 keys far from zero (minVal = -2^40 - 7) over R = 2^10: a single
    tile with 32-bit counters in every piece."""
    n, lo, R = 2 * PIECE + (1 << 20) + 1, -(1 << 40) - 7, 1 << 10
    _say(f"int64 n={n} minVal={lo} R={R}")
    a = _uniform(n, lo, lo + R, inputs.case_seed(72, R), torch.int64)
    _plant(a, [(lo, 2), (lo + R - 1, 3)])
    cnt = _counts(a, lo, R)
    b = torch.empty_like(a)
    r.sort_keys(a, lo, lo + R, keys_out=b)
    torch.cuda.synchronize()
    del a
    _verify(b, cnt, lo, n)


def test_int32_wide_workspace_in_place(r):
    """The caller-workspace form, in place, at R = 2^22 (27 LDS passes, so
    every piece is first partitioned by pass): rtcdf_workspace_bytes gives
    the size, one byte less is refused before any GPU work."""
    n, lo, R = 2 * PIECE + 7, 1 << 20, 1 << 22
    _say(f"int32 n={n} R={R} in place, caller workspace")
    a = _uniform(n, lo, lo + R, inputs.case_seed(73, R), torch.int32)
    cnt = _counts(a, lo, R)
    need = r.workspace_bytes(n, lo, lo + R, keys_out=a)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    with pytest.raises(r.RtcdfError) as e:
        r.sort_ws(a, a, lo, lo + R, ws[:need - 1])
    assert e.value.status == r.WORKSPACE_TOO_SMALL
    r.sort_ws(a, a, lo, lo + R, ws)
    torch.cuda.synchronize()
    del ws
    _verify(a, cnt, lo, n)
