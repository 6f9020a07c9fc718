"""The multi-threaded CPU counting sort that the benchmark times beside the
oracle is checked against the oracle (Sec. 2.1 sort), element by element, on
random, skewed, degenerate and ragged inputs over several thread counts."""
import numpy as np
import pytest

import oracle

I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1


@pytest.mark.parametrize("threads", [1, 2, 3, 8, 17])
@pytest.mark.parametrize("n,R,dist", [
    (0, 5, "uniform"), (1, 1, "uniform"), (7, 3, "uniform"), (1000, 1, "uniform"),
    (100003, 4096, "uniform"), (100003, 70000, "uniform"), (50000, 1 << 18, "sparse"),
    (200001, 1024, "zipf"), (99999, 513, "one_value"),
])
def test_matches_oracle(threads, n, R, dist):
    rng = np.random.default_rng(n * 31 + R + threads)
    minVal = -12345
    if dist == "uniform":
        x = rng.integers(0, R, n)
    elif dist == "sparse":
        x = rng.choice(rng.integers(0, R, 17), n)
    elif dist == "zipf":
        x = np.minimum(rng.zipf(1.3, n) - 1, R - 1)
    else:
        x = np.full(n, R // 2)
    A = (x + minVal).astype(np.int32)
    B, used = oracle.parallel_sort(A, minVal, minVal + R, threads)
    assert 1 <= used <= max(1, threads)
    assert np.array_equal(B, oracle.sort(A, minVal, minVal + R))


def test_full_int32_edges():
    # keys at both ends of int32; the range's upper end is INT32_MAX + 1
    A = np.array([I32_MAX, I32_MAX - 3, I32_MAX, I32_MAX - 1] * 1000, dtype=np.int32)
    B, _ = oracle.parallel_sort(A, I32_MAX - 3, I32_MAX + 1, 4)
    assert np.array_equal(B, oracle.sort(A, I32_MAX - 3, I32_MAX + 1))
    A = np.array([I32_MIN + 1, I32_MIN] * 777, dtype=np.int32)
    B, _ = oracle.parallel_sort(A, I32_MIN, I32_MIN + 2, 3)
    assert np.array_equal(B, oracle.sort(A, I32_MIN, I32_MIN + 2))


def test_fewer_keys_than_threads():
    A = np.array([5, 3, 4], dtype=np.int32)
    B, used = oracle.parallel_sort(A, 3, 6, 16)
    assert used == 3 and B.tolist() == [3, 4, 5]


@pytest.mark.parametrize("bad_key", [-1, 10])
def test_key_out_of_range(bad_key):
    A = np.arange(10000, dtype=np.int32) % 10
    A[7777] = bad_key
    with pytest.raises(oracle.OracleError) as e:
        oracle.parallel_sort(A, 0, 10, 4)
    assert e.value.code == oracle.ORC_KEY_OUT_OF_RANGE


@pytest.mark.parametrize("lo,hi,threads", [(5, 5, 2), (6, 5, 2), (0, 1 << 33, 2), (0, 4, 0)])
def test_invalid_arguments(lo, hi, threads):
    with pytest.raises(oracle.OracleError) as e:
        oracle.parallel_sort(np.zeros(4, dtype=np.int32), lo, hi, threads)
    assert e.value.code == oracle.ORC_INVALID_ARGUMENT
