"""Reference (CPU, float64) for the learned configuration picker -- TEST
INFRASTRUCTURE ONLY: used by the tests to check the HIP kernels, never by the
product library.

The picker predicts, from features of an input array, the runtime of every
kernel configuration of the sort and picks the fastest valid one.  Each
function below is the plain definition of one step, written out:

  sketch      features of an array: log2 n, log2 R and the fractions of S
              evenly spaced sample keys that fall in each of B equal-width
              bins of the range (bin = floor((key - minVal) * B / R));
  forward     a fully connected network with ReLU hidden layers,
              y = W3 relu(W2 relu(W1 x + b1) + b2) + b3;
  loss        masked mean squared error over the valid configurations,
              L = sum(M (y - t)^2) / sum(M);
  backward    gradients of L by the chain rule;
  adam_step   the Adam update of Kingma and Ba (2015): moments m, v with
              decay rates beta1, beta2, bias correction by 1 - beta^t, step
              -lr * mhat / (sqrt(vhat) + eps);
  pick        argmin of the prediction over the valid configurations
              (lowest index on ties).

Parity pins live in tests/test_mlp_ref.py.
"""
from __future__ import annotations

import numpy as np


def sketch(keys: np.ndarray, minVal: int, maxVal: int, samples: int = 4096, bins: int = 32):
    """[log2 n, log2 R, frac_0 .. frac_{bins-1}] of the keys.  Sample i is the
    key at position floor(i * n / S) for i < S, with S = min(samples, n)."""
    keys = np.asarray(keys)
    n = keys.size
    R = int(maxVal) - int(minVal)
    S = min(int(samples), n)
    counts = [0] * bins
    for i in range(S):
        key = int(keys[(i * n) // S])
        b = ((key - int(minVal)) * bins) // R
        counts[b] += 1
    feats = [np.log2(n) if n > 0 else 0.0, np.log2(R)]
    feats += [c / S if S else 0.0 for c in counts]
    return np.array(feats, dtype=np.float64)


def relu(z):
    return np.maximum(z, 0.0)


def forward(params, X):
    """X: (batch, d_in).  Returns (Y, cache)."""
    W1, b1, W2, b2, W3, b3 = (params[k] for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    Z1 = X @ W1.T + b1
    H1 = relu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = relu(Z2)
    Y = H2 @ W3.T + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss(Y, T, M):
    return float(np.sum(M * (Y - T) ** 2) / np.sum(M))


def backward(params, cache, Y, T, M):
    """Gradients of the masked MSE with respect to every parameter."""
    X, Z1, H1, Z2, H2 = cache
    dY = 2.0 * M * (Y - T) / np.sum(M)
    g = {}
    g["W3"] = dY.T @ H2
    g["b3"] = dY.sum(axis=0)
    dH2 = dY @ params["W3"]
    dZ2 = dH2 * (Z2 > 0)
    g["W2"] = dZ2.T @ H1
    g["b2"] = dZ2.sum(axis=0)
    dH1 = dZ2 @ params["W2"]
    dZ1 = dH1 * (Z1 > 0)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1).  Updates params, m, v in place."""
    for k in params:
        m[k] = beta1 * m[k] + (1.0 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * grads[k] ** 2
        mhat = m[k] / (1.0 - beta1 ** t)
        vhat = v[k] / (1.0 - beta2 ** t)
        params[k] = params[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return params, m, v


def pick(Y, valid):
    """Index of the smallest prediction among the valid configurations."""
    best, arg = None, -1
    for j in range(len(valid)):
        if valid[j] and (best is None or Y[j] < best):
            best, arg = Y[j], j
    return arg
