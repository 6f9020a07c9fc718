"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: the worked example of
Sec. 3.1, the H-P example of Sec. 2.2, a library sort by brute force on every
tiny array, independent counting routes for the invariants of Lemmas 1-3 and
Theorem 1, and special cases whose answer is known in closed form.
"""
import itertools

import numpy as np
import pytest

import oracle
from tests.golden.load import load

I32_MIN = -(2 ** 31)


def test_worked_example_tiles():
    g = load("worked_example.txt")
    hist, cdf, O = oracle.tile_intermediates(g["A"], g["minVal"], g["maxVal"], g["T"])
    assert hist.tolist() == g["hist"].tolist()
    assert cdf.tolist() == g["cdf"].tolist()
    assert O.tolist() == g["O"].tolist()
    B = oracle.output_from_local_cdfs(cdf, O, g["minVal"], g["maxVal"], g["T"], g["A"].size)
    assert B.tolist() == g["B"].tolist()
    assert oracle.sort(g["A"], g["minVal"], g["maxVal"]).tolist() == g["B"].tolist()


def test_hp_example():
    g = load("hp_example.txt")
    A = np.repeat(np.arange(g["counts"].size), g["counts"])
    A = A[np.random.default_rng(5).permutation(A.size)]
    cnt = oracle.counts(A, g["minVal"], g["maxVal"])
    assert cnt.tolist() == g["counts"].tolist()
    P1 = np.cumsum(cnt)
    assert P1.tolist() == g["P1"].tolist()
    assert oracle.prefix_max_output(P1, g["minVal"], g["maxVal"], A.size).tolist() == g["B"].tolist()
    assert oracle.sort(A, g["minVal"], g["maxVal"]).tolist() == g["B"].tolist()


@pytest.mark.parametrize("R", [1, 2, 3, 4])
def test_exhaustive_tiny_vs_library_sort(R):
    """Every array of length <= 6 over a range of R values, at three offsets."""
    for minVal in (0, -3, I32_MIN):
        maxVal = minVal + R
        for n in range(0, 7):
            for tup in itertools.product(range(R), repeat=n):
                A = np.array(tup, dtype=np.int64) + minVal
                want = sorted(A.tolist())
                assert oracle.sort(A, minVal, maxVal).tolist() == want
                for T in range(1, R + 1):
                    _, cdf, O = oracle.tile_intermediates(A, minVal, maxVal, T)
                    got = oracle.output_from_local_cdfs(cdf, O, minVal, maxVal, T, n)
                    assert got.tolist() == want


def _direct_lemmas(A, minVal, maxVal, T, hist, cdf, O):
    """Lemmas 1 and 2 by direct counting over the keys (no prefix sums)."""
    R = maxVal - minVal
    x = A.astype(np.int64) - minVal
    m = -(-R // T)
    for t in range(m):
        b = t * T
        w = min(T, R - b)
        assert O[t] == np.count_nonzero(x < b)                    # Lemma 2
        for j in range(w):
            assert hist[b + j] == np.count_nonzero(x == b + j)    # Alg. 5
            assert cdf[b + j] == np.count_nonzero((x >= b) & (x <= b + j))  # Lemma 1


@pytest.mark.parametrize("seed", range(6))
def test_random_small_lemmas(seed):
    rng = np.random.default_rng(seed)
    R = int(rng.integers(1, 70))
    minVal = int(rng.integers(-10 ** 6, 10 ** 6))
    n = int(rng.integers(0, 300))
    A = rng.integers(minVal, minVal + R, size=n)
    for T in sorted({1, 2, 3, 7, 16, R, R + 5}):
        hist, cdf, O = oracle.tile_intermediates(A, minVal, minVal + R, T)
        _direct_lemmas(A, minVal, minVal + R, T, hist, cdf, O)


@pytest.mark.parametrize("seed", range(8))
def test_random_medium_vs_numpy_sort(seed):
    rng = np.random.default_rng(100 + seed)
    R = int(rng.integers(1, 1 << 12))
    minVal = int(rng.integers(-2 ** 31, 2 ** 31 - R))
    n = int(rng.integers(0, 20000))
    A = rng.integers(minVal, minVal + R, size=n)
    B = oracle.sort(A, minVal, minVal + R)
    assert np.array_equal(B, np.sort(A).astype(np.int32))
    # Theorem 1 invariants, checked without the sort:
    assert np.all(np.diff(B.astype(np.int64)) >= 0)
    assert np.array_equal(np.bincount(B.astype(np.int64) - minVal, minlength=R),
                          np.bincount(A - minVal, minlength=R))
    assert B.astype(np.int64).sum() == A.sum()
    # Lemma 3: value v occupies [#keys < v, #keys <= v)
    for v in rng.integers(minVal, minVal + R, size=20):
        lo, hi = np.count_nonzero(A < v), np.count_nonzero(A <= v)
        assert np.all(B[lo:hi] == v)
        assert (lo == 0 or B[lo - 1] < v) and (hi == n or B[hi] > v)
    # the tiled method reaches the same array for several tile widths
    for T in (1, 5, 64, 1000, R):
        _, cdf, O = oracle.tile_intermediates(A, minVal, minVal + R, T)
        assert np.array_equal(oracle.output_from_local_cdfs(cdf, O, minVal, minVal + R, T, n), B)
    # Alg. 3 on the full-range CDF reaches it too
    P1 = np.cumsum(oracle.counts(A, minVal, minVal + R))
    if n > 0:
        assert np.array_equal(oracle.prefix_max_output(P1, minVal, minVal + R, n), B)


def test_special_cases():
    rng = np.random.default_rng(7)
    # all equal -> output equals the input
    A = np.full(1000, 42, dtype=np.int32)
    assert np.array_equal(oracle.sort(A, 0, 128), A)
    # already sorted -> itself; reverse sorted -> reversed
    A = np.sort(rng.integers(-50, 50, size=777))
    assert np.array_equal(oracle.sort(A, -50, 50), A)
    assert np.array_equal(oracle.sort(A[::-1], -50, 50), A)
    # R = 1
    A = np.full(10, -7)
    assert np.array_equal(oracle.sort(A, -7, -6), A)
    # n = 0
    assert oracle.sort(np.zeros(0, dtype=np.int32), 0, 10).size == 0
    # extreme ends of int32: [INT32_MIN, INT32_MIN + 5) and [2^31 - 5, 2^31)
    A = rng.integers(I32_MIN, I32_MIN + 5, size=100)
    assert np.array_equal(oracle.sort(A, I32_MIN, I32_MIN + 5), np.sort(A))
    A = rng.integers(2 ** 31 - 5, 2 ** 31, size=100)
    assert np.array_equal(oracle.sort(A, 2 ** 31 - 5, 2 ** 31), np.sort(A))
    # full int32 range is a legal (if huge) range for counts of a tiny array
    # is not exercised: R = 2^32 counters would need 32 GiB.


def test_errors():
    with pytest.raises(oracle.OracleError) as e:
        oracle.sort(np.array([0, 1, 5]), 0, 5)
    assert e.value.code == oracle.ORC_KEY_OUT_OF_RANGE
    with pytest.raises(oracle.OracleError) as e:
        oracle.sort(np.array([-1]), 0, 5)
    assert e.value.code == oracle.ORC_KEY_OUT_OF_RANGE
    for lo, hi in ((5, 5), (6, 5), (I32_MIN - 1, 0), (0, 2 ** 31 + 1)):
        with pytest.raises(oracle.OracleError) as e:
            oracle.counts(np.zeros(0, dtype=np.int32), lo, hi)
        assert e.value.code == oracle.ORC_INVALID_ARGUMENT


def test_streaming_verifier():
    rng = np.random.default_rng(11)
    minVal, R = -300, 1000
    A = rng.integers(minVal, minVal + R, size=50000)
    cnt = oracle.counts(A, minVal, minVal + R)
    B = np.sort(A).astype(np.int32)
    v = oracle.StreamingVerifier(cnt, minVal)
    pos = 0
    while pos < B.size:
        k = int(rng.integers(1, 5000))
        v.chunk(B[pos:pos + k])
        pos += k
    v.end(B.size)
    # a single wrong element is found at its position
    for bad in (0, 1234, B.size - 1):
        C = B.copy()
        C[bad] = C[bad] + 1 if C[bad] < minVal + R - 1 else C[bad] - 1
        v = oracle.StreamingVerifier(cnt, minVal)
        with pytest.raises(oracle.OracleError, match=f"position {bad}"):
            v.chunk(C[:30000])
            v.chunk(C[30000:])
    # too short / too long
    v = oracle.StreamingVerifier(cnt, minVal)
    v.chunk(B[:-1])
    with pytest.raises(oracle.OracleError):
        v.end(B.size)
    v = oracle.StreamingVerifier(cnt, minVal)
    with pytest.raises(oracle.OracleError):
        v.chunk(np.concatenate([B, B[-1:]]))


def test_streaming_verifier_counts_over_2pow32():
    """The verifier's cursor is 64-bit (sorts of n >= 2^32 keys): one value
    held 2^32 + 5 times, then three copies of the next, fed in chunks of one
    reused 2^24-key array.  A wrong element at position 2^32 + 4 (the last
    copy of the first value) is reported at that position, which neither a
    32-bit count nor a 32-bit position could hold."""
    minVal, big = -3, (1 << 32) + 5
    cnt = np.array([big, 3], dtype=np.uint64)
    run = np.full(1 << 24, minVal, dtype=np.int32)

    def feed(v, upto):
        for _ in range(upto >> 24):
            v.chunk(run)
        v.chunk(run[:upto & ((1 << 24) - 1)])

    v = oracle.StreamingVerifier(cnt, minVal)
    feed(v, big)
    v.chunk(np.full(3, minVal + 1, dtype=np.int32))
    v.end(big + 3)
    assert v.position == big + 3
    v = oracle.StreamingVerifier(cnt, minVal)
    feed(v, big - 1)
    with pytest.raises(oracle.OracleError, match=f"position {big - 1}"):
        v.chunk(np.array([minVal + 1], dtype=np.int32))


@pytest.mark.parametrize("seed", range(4))
def test_sparse_and_offset_keys(seed):
    """Keys that avoid the low and high ends of the declared range, with long runs
    of absent values between them: the step writes of Alg. 3 then start at a value
    above minVal, and Alg. 7 must skip empty bins and empty tiles."""
    rng = np.random.default_rng(300 + seed)
    minVal, R = int(rng.integers(-1000, 1000)), int(rng.integers(50, 3000))
    present = rng.choice(np.arange(3, R - 3), size=int(rng.integers(1, 8)), replace=False)
    A = minVal + rng.choice(present, size=int(rng.integers(2, 500)))
    want = np.sort(A).astype(np.int32)
    assert np.array_equal(oracle.sort(A, minVal, minVal + R), want)
    P1 = np.cumsum(oracle.counts(A, minVal, minVal + R))
    assert np.array_equal(oracle.prefix_max_output(P1, minVal, minVal + R, A.size), want)
    for T in (1, 4, 33, R):
        _, cdf, O = oracle.tile_intermediates(A, minVal, minVal + R, T)
        assert np.array_equal(oracle.output_from_local_cdfs(cdf, O, minVal, minVal + R, T, A.size), want)
