"""GPU parity of the sort of 16- and 8-bit keys (rtcdf_sort_keys) against the
CPU oracle, which sorts the same keys widened to int32: ragged n with every
input/output misalignment within a 16-byte vector, full and partial ranges
(single-tile fast path and staged path), four distributions, in place,
several configurations, and 10^8 keys checked by the streaming verifier."""
import sys

import numpy as np
import pytest

import oracle
from paper_2609_00843_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TYPES = {"int16": (np.int16, -32768, 32768), "uint16": (np.uint16, 0, 65536),
         "int8": (np.int8, -128, 128), "uint8": (np.uint8, 0, 256)}
_VIEW = {np.uint16: (np.int16, "uint16")}


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def r():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_00843_amd import rtcdf
    return rtcdf


def _tdtype(npt):
    return {np.int16: torch.int16, np.uint16: torch.uint16, np.int8: torch.int8, np.uint8: torch.uint8}[npt]


def _to_dev(A, npt, pad, fill):
    """Device buffer with A at element offset `pad`, the rest `fill`."""
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


def _check(r, A, npt, lo, hi, pin=0, pout=0, inplace=False, cfg=None):
    _say(f"keys {npt.__name__} n={A.size} [{lo},{hi}) pin={pin} pout={pout} inplace={inplace} cfg={cfg}")
    want = oracle.sort(A.astype(np.int32), lo, hi).astype(npt)
    bin_, tin = _to_dev(A, npt, pin, 7)
    if inplace:
        r.sort_keys(tin, lo, hi, keys_out=tin, config=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(_to_host(tin, npt), want)
        return
    bout, tout = _to_dev(np.zeros(A.size, dtype=npt), npt, pout, 0x5A)
    r.sort_keys(tin, lo, hi, keys_out=tout, config=cfg)
    torch.cuda.synchronize()
    got = _to_host(tout, npt)
    assert np.array_equal(got, want), f"mismatch at {np.flatnonzero(got != want)[:8]}"
    full = _to_host(bout, npt)
    guard = np.array(0x5A, dtype=npt)
    assert np.all(full[:pout] == guard) and np.all(full[pout + A.size:] == guard)
    assert np.array_equal(_to_host(tin, npt), A)


@pytest.mark.parametrize("name", list(TYPES))
def test_ragged_and_misaligned(r, name):
    npt, tlo, thi = TYPES[name]
    rng = np.random.default_rng(len(name))
    for i, n in enumerate((1, 2, 3, 7, 15, 16, 17, 33, 1023, 4099, 65537, 300001)):
        for lo, hi in ((tlo, thi), (tlo + 3, tlo + 3 + min(200, thi - tlo - 3)), (thi - 1, thi)):
            A = rng.integers(lo, hi, size=n).astype(npt)
            _check(r, A, npt, lo, hi, pin=i % 16, pout=(3 * i + 5) % 16)


@pytest.mark.parametrize("name", list(TYPES))
@pytest.mark.parametrize("dist", ["uniform", "normal", "all_equal", "zipf"])
def test_distributions(r, name, dist):
    npt, tlo, thi = TYPES[name]
    A = (inputs.make(dist, 2_000_003, 0, thi - tlo, 17).astype(np.int64) + tlo).astype(npt)
    _check(r, A, npt, tlo, thi, pout=1)


@pytest.mark.parametrize("name", ["int16", "uint8"])
def test_in_place_and_configs(r, name):
    npt, tlo, thi = TYPES[name]
    rng = np.random.default_rng(5)
    A = rng.integers(tlo, thi, size=500_001).astype(npt)
    _check(r, A, npt, tlo, thi, inplace=True)
    for T, items, bpt in ((128, 4, 4), (1024, 8, 2), (8192, 16, 1), (32768, 4, 1)):
        _check(r, A, npt, tlo, thi, cfg=r.make_config(T, items, bpt), pin=2, pout=3)


@pytest.mark.parametrize("name", ["int16", "uint8"])
def test_full_size(r, name):
    """10^8 keys over the type's whole range, compared with the oracle's counts."""
    npt, tlo, thi = TYPES[name]
    n = 10 ** 8
    rng = np.random.default_rng(9)
    A = rng.integers(tlo, thi, size=n).astype(npt)
    _say(f"keys full size {name}")
    tin = torch.from_numpy(A).cuda()
    out = r.sort_keys(tin, tlo, thi)
    torch.cuda.synchronize()
    cnt = oracle.counts(A.astype(np.int32), tlo, thi)
    v = oracle.StreamingVerifier(cnt, tlo)
    for i in range(0, n, 1 << 25):
        v.chunk(out[i:i + (1 << 25)].cpu().numpy().astype(np.int32))
    v.end(n)


@pytest.mark.parametrize("sub", [0, 1, 4])
@pytest.mark.parametrize("name,lo,hi", [("uint8", 0, 256), ("int8", -128, 128), ("int16", -1000, 1048),
                                        ("uint16", 7, 1500)])
def test_counter_copies(r, monkeypatch, sub, name, lo, hi):
    """LDS copies of the 32-bit counters (none, 2 or 16 per bin; 8-bit keys
    take 8 by default) on narrow keys: single-tile fast path and staged path,
    ragged n with head and tail keys, skewed and uniform values."""
    npt = TYPES[name][0]
    monkeypatch.setenv("RTCDF_DEV_HIST_SPREAD", str(sub))
    rng = np.random.default_rng(sub * 7 + len(name))
    for fast in ("1", "0"):
        monkeypatch.setenv("RTCDF_DEV_FAST", fast)
        for n in (300_007, 1_000_001):
            x = rng.integers(lo, hi, size=n)
            x[: n // 3] = lo + (hi - lo) // 3            # a third of the keys on one value
            _check(r, x.astype(npt), npt, lo, hi, pin=3, pout=5)


def test_sort_dispatches_by_dtype(r):
    """rtcdf.sort takes narrow key tensors too (through rtcdf_sort_keys)."""
    rng = np.random.default_rng(2)
    A = rng.integers(-300, 300, size=100_003).astype(np.int16)
    _say("sort() with int16 keys")
    out = r.sort(torch.from_numpy(A).cuda(), -300, 300)
    torch.cuda.synchronize()
    assert out.dtype == torch.int16
    assert np.array_equal(out.cpu().numpy(), oracle.sort(A.astype(np.int32), -300, 300).astype(np.int16))


# ---- int64 keys (rtcdf_sort_keys, RTCDF_KEY_INT64) ----------------------------

I64MIN, I64MAX = -(1 << 63), (1 << 63) - 1


def _want64(A, lo, hi):
    """The oracle's sort of the normalised values key - lo (Sec. 2.1: minVal is
    notation; the counting sort is the same on [0, R)), shifted back; checked
    against numpy's sort as a second, independent reference."""
    R = hi - lo
    x = (A.astype(object) - lo).astype(np.int64) if lo < -(1 << 62) else (A - np.int64(lo))
    want = oracle.sort(x.astype(np.int32), 0, R).astype(np.int64)
    want = (want.astype(object) + lo).astype(np.int64) if lo < -(1 << 62) else want + np.int64(lo)
    assert np.array_equal(want, np.sort(A))
    return want


def _check64(r, A, lo, hi, pin=0, pout=0, inplace=False, cfg=None):
    _say(f"int64 keys n={A.size} [{lo},{hi}) pin={pin} pout={pout} inplace={inplace} cfg={cfg}")
    want = _want64(A, lo, hi)
    buf = np.full(A.size + pin + 4, 7, dtype=np.int64)
    buf[pin:pin + A.size] = A
    tb = torch.from_numpy(buf).cuda()
    tin = tb[pin:pin + A.size]
    if inplace:
        r.sort_keys(tin, lo, hi, keys_out=tin, config=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(tin.cpu().numpy(), want)
        return
    bout = torch.full((A.size + pout + 4,), 0x5A5A5A5A5A5A5A5A, dtype=torch.int64, device="cuda")
    tout = bout[pout:pout + A.size]
    r.sort_keys(tin, lo, hi, keys_out=tout, config=cfg)
    torch.cuda.synchronize()
    got = tout.cpu().numpy()
    assert np.array_equal(got, want), f"mismatch at {np.flatnonzero(got != want)[:8]}"
    full = bout.cpu().numpy()
    assert np.all(full[:pout] == 0x5A5A5A5A5A5A5A5A) and np.all(full[pout + A.size:] == 0x5A5A5A5A5A5A5A5A)
    assert np.array_equal(tin.cpu().numpy(), A)


@pytest.mark.parametrize("lo,R", [(0, 1), (-5, 7), (10 ** 12, 128), (-(10 ** 15), 2048), (3, 2049),
                                  (I64MIN, 65536), (I64MAX - (1 << 18), 1 << 18), (-(1 << 40), 1 << 20)])
def test_int64_ragged_and_misaligned(r, lo, R):
    """Ragged n with both 8-byte alignments of input and output inside a
    16-byte vector, windows anywhere in the int64 values (both extremes), the
    single-tile fast path (R <= 2048) and the staged path."""
    rng = np.random.default_rng(R)
    for i, n in enumerate((1, 2, 3, 4, 5, 7, 9, 1023, 4099, 65537, 300001)):
        x = rng.integers(0, R, size=n)
        A = np.array([lo + int(v) for v in x], dtype=np.int64) if lo < -(1 << 62) else x.astype(np.int64) + np.int64(lo)
        _check64(r, A, lo, lo + R, pin=i % 2, pout=(i // 2) % 2)


@pytest.mark.parametrize("dist", ["uniform", "normal", "all_equal", "zipf"])
@pytest.mark.parametrize("R", [1 << 10, 1 << 16, 1 << 18])
def test_int64_distributions(r, dist, R):
    lo = 7 * 10 ** 14
    A = inputs.make(dist, 2_000_003, 0, R, 23).astype(np.int64) + np.int64(lo)
    _check64(r, A, lo, lo + R, pout=1)


def test_int64_in_place_and_configs(r):
    rng = np.random.default_rng(6)
    lo = -(10 ** 13)
    A = rng.integers(0, 1 << 17, size=700_001).astype(np.int64) + np.int64(lo)
    _check64(r, A, lo, lo + (1 << 17), inplace=True)
    for T, items, bpt in ((128, 4, 4), (1024, 8, 2), (8192, 16, 1), (32768, 4, 1)):
        _check64(r, A, lo, lo + (1 << 17), cfg=r.make_config(T, items, bpt), pin=1, pout=0)


@pytest.mark.parametrize("sub", [1, 4])
def test_int64_counter_copies(r, monkeypatch, sub):
    """LDS copies of the 32-bit counters with int64 keys (two keys per
    16-byte vector), fast and staged paths."""
    monkeypatch.setenv("RTCDF_DEV_HIST_SPREAD", str(sub))
    rng = np.random.default_rng(sub)
    lo, R = -(1 << 40) + 11, 1000
    for fast in ("1", "0"):
        monkeypatch.setenv("RTCDF_DEV_FAST", fast)
        A = rng.integers(0, R, size=500_003).astype(np.int64) + np.int64(lo)
        _check64(r, A, lo, lo + R, pin=1, pout=0)


def test_int64_full_size(r):
    """5 x 10^7 int64 keys over 2^18 values, compared with the oracle's counts
    by the streaming verifier."""
    n, lo, R = 50_000_000, 123_456_789_012, 1 << 18
    rng = np.random.default_rng(10)
    x = rng.integers(0, R, size=n).astype(np.int32)
    _say("int64 keys full size")
    tin = torch.from_numpy(x.astype(np.int64) + np.int64(lo)).cuda()
    out = r.sort(tin, lo, lo + R)
    torch.cuda.synchronize()
    assert out.dtype == torch.int64
    cnt = oracle.counts(x, 0, R)
    v = oracle.StreamingVerifier(cnt, 0)
    for i in range(0, n, 1 << 24):
        v.chunk((out[i:i + (1 << 24)] - lo).to(torch.int32).cpu().numpy())
    v.end(n)
