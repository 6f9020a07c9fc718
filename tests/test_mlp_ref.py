"""Pins for the float64 reference of the learned picker (no GPU): backward
against central finite differences of forward, forward and loss against
hand-computed values, Adam against its closed-form first step and a
convergence check, the sketch against closed-form cases, pick against
special cases."""
import numpy as np
import pytest

from oracle import mlp_ref as M


def _params(rng, sizes):
    p = {}
    for i in range(3):
        p[f"W{i + 1}"] = rng.normal(0, 1.0 / np.sqrt(sizes[i]), size=(sizes[i + 1], sizes[i]))
        p[f"b{i + 1}"] = rng.normal(0, 0.1, size=sizes[i + 1])
    return p


@pytest.mark.parametrize("sizes", [(5, 4, 3, 2), (34, 64, 64, 62)])
def test_backward_matches_finite_differences(sizes):
    rng = np.random.default_rng(sum(sizes))
    p = _params(rng, sizes)
    X = rng.normal(size=(7, sizes[0]))
    T = rng.normal(size=(7, sizes[-1]))
    Mk = (rng.random(size=(7, sizes[-1])) < 0.8).astype(np.float64)
    Y, cache = M.forward(p, X)
    g = M.backward(p, cache, Y, T, Mk)
    eps = 1e-6
    for k, W in p.items():
        idx = [tuple(rng.integers(0, s) for s in W.shape) for _ in range(6)]
        for ix in idx:
            old = W[ix]
            W[ix] = old + eps
            lp = M.loss(M.forward(p, X)[0], T, Mk)
            W[ix] = old - eps
            lm = M.loss(M.forward(p, X)[0], T, Mk)
            W[ix] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[k][ix]) <= 1e-6 * max(1.0, abs(fd)), (k, ix, fd, g[k][ix])


def test_forward_and_loss_by_hand():
    p = {"W1": np.array([[1.0, -1.0]]), "b1": np.array([0.5]),
         "W2": np.array([[2.0]]), "b2": np.array([-1.0]),
         "W3": np.array([[3.0]]), "b3": np.array([1.0])}
    Y, _ = M.forward(p, np.array([[2.0, 1.0], [0.0, 1.0]]))
    # (2,1): relu(1.5)=1.5 -> relu(2)=2 -> 7 ; (0,1): relu(-0.5)=0 -> relu(-1)=0 -> 1
    assert Y[:, 0].tolist() == [7.0, 1.0]
    T = np.array([[5.0], [4.0]])
    assert M.loss(Y, T, np.array([[1.0], [1.0]])) == pytest.approx((4 + 9) / 2)
    assert M.loss(Y, T, np.array([[0.0], [1.0]])) == pytest.approx(9.0)


def test_adam_first_step_and_convergence():
    # With zero moments, the bias-corrected first step is -lr * g / (|g| + eps).
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    M.adam_step(p, g, m, v, 1, lr=0.1)
    want = np.array([1.0, -2.0, 3.0]) - 0.1 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], want, rtol=0, atol=1e-12)
    # minimises (w - 3)^2
    p = {"w": np.array([0.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    for t in range(1, 3001):
        M.adam_step(p, {"w": 2 * (p["w"] - 3.0)}, m, v, t, lr=0.05)
    assert abs(p["w"][0] - 3.0) < 1e-3


def test_sketch_closed_forms():
    # all keys equal -> one bin holds everything
    f = M.sketch(np.full(10000, 7, dtype=np.int32), 0, 64, samples=4096, bins=32)
    assert f[0] == pytest.approx(np.log2(10000)) and f[1] == pytest.approx(6.0)
    assert f[2 + 3] == 1.0 and f[2:].sum() == 1.0
    # every value of R = 64 equally often, sampled exactly -> 2 values per bin, all 1/32
    keys = np.tile(np.arange(-10, 54, dtype=np.int32), 64)       # n = 4096, sample i -> key i
    f = M.sketch(keys, -10, 54, samples=4096, bins=32)
    assert np.allclose(f[2:], 1.0 / 32)
    # bin boundaries: key minVal + ceil(j * R / B) is the first key of bin j (R = 100, B = 32)
    R, B = 100, 32
    for j in range(B):
        first = -(-(j * R) // B)
        f = M.sketch(np.array([5 + first], dtype=np.int32), 5, 5 + R, samples=8, bins=B)
        assert f[2 + j] == 1.0
    # fewer keys than samples: every key is sampled once
    f = M.sketch(np.array([0, 99, 99], dtype=np.int32), 0, 100, samples=4096, bins=4)
    assert np.allclose(f[2:], [1 / 3, 0, 0, 2 / 3])


def test_pick():
    assert M.pick(np.array([3.0, 1.0, 1.0, 0.5]), [True, True, True, False]) == 1
    assert M.pick(np.array([3.0, 2.0]), [False, True]) == 1
    assert M.pick(np.array([3.0, 2.0]), [False, False]) == -1
