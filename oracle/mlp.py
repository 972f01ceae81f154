"""Per-pair features and the warm-start MLP, plain FP64 definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).  These are the
reference definitions that the GPU feature, forward, backward and Adam
kernels are checked against.

Features of pair g (strong orbital s = g, weak orbitals w_0.. in ascending
index, padded to KMAX = 6 slots; mean field m_x = sum over the other strong
orbitals t of (2 J_xt - K_xt)):
    [H_ss, J_ss, m_s] + per slot k: [H_ww - H_ss, J_ww, K_sw, J_sw, m_w] + 6 slot masks
    (39 values; empty slots are zero).
Targets: the pair's converged ONs [n_s, n_w0, .., n_w5] (7 values, mask
[1, slot masks]).

Network: 39 -> 128 -> 128 -> 128 -> 7, tanh hidden activations, masked
softmax output p (empty slots get p = 0), loss = mean over rows of
sum_k mask_k (p_k - t_k)^2.  Parameters are one flat vector
[W1 (39x128), b1, W2 (128x128), b2, W3 (128x128), b3, W4 (128x7), b4], each W
row-major [in][out] (y = x W + b).
"""
from __future__ import annotations

import numpy as np

from .on_opt import weak_lists

KMAX = 6
N_IN = 3 + 5 * KMAX + KMAX   # 39
N_HID = 128
N_OUT = 1 + KMAX             # 7
SHAPES = [(N_IN, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID, N_OUT), (N_OUT,)]
N_PARAMS = int(sum(np.prod(s) for s in SHAPES))

__all__ = ["KMAX", "N_IN", "N_HID", "N_OUT", "N_PARAMS", "features", "targets", "unpack", "init_params",
           "forward", "backward", "loss", "adam_step"]


def features(Hpp, J, K, pair_of, n_pairs, n_cwo):
    weak = weak_lists(pair_of, n_pairs)
    X = np.zeros((n_pairs, N_IN))

    def mf(x, s):
        return sum(2.0 * J[x, t] - K[x, t] for t in range(n_pairs) if t != s)

    for g in range(n_pairs):
        s = g
        X[g, 0], X[g, 1], X[g, 2] = Hpp[s], J[s, s], mf(s, s)
        for k, w in enumerate(weak[g][:KMAX]):
            X[g, 3 + 5 * k: 8 + 5 * k] = [Hpp[w] - Hpp[s], J[w, w], K[s, w], J[s, w], mf(w, s)]
            X[g, 3 + 5 * KMAX + k] = 1.0
    return X


def targets(n, pair_of, n_pairs):
    weak = weak_lists(pair_of, n_pairs)
    T = np.zeros((n_pairs, N_OUT))
    M = np.zeros((n_pairs, N_OUT))
    for g in range(n_pairs):
        T[g, 0], M[g, 0] = n[g], 1.0
        for k, w in enumerate(weak[g][:KMAX]):
            T[g, 1 + k], M[g, 1 + k] = n[w], 1.0
    return T, M


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        size = int(np.prod(s))
        out.append(theta[o:o + size].reshape(s))
        o += size
    return out


def init_params(seed=0):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            a = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-a, a, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def forward(theta, X, M):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    h3 = np.tanh(h2 @ W3 + b3)
    z = h3 @ W4 + b4
    zm = np.where(M > 0, z, -np.inf)
    zmax = np.max(zm, axis=1, keepdims=True)
    e = np.where(M > 0, np.exp(z - zmax), 0.0)
    p = e / np.sum(e, axis=1, keepdims=True)
    return p, (X, h1, h2, h3, p)


def loss(p, T, M):
    return float(np.sum(M * (p - T) ** 2) / p.shape[0])


def backward(theta, cache, T, M):
    """Gradient of loss() with respect to theta (same flat layout)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    X, h1, h2, h3, p = cache
    N = X.shape[0]
    dp = 2.0 * M * (p - T) / N
    dz = p * (dp - np.sum(dp * p, axis=1, keepdims=True))      # softmax Jacobian (p = 0 off-mask)
    gW4, gb4 = h3.T @ dz, dz.sum(0)
    d3 = (dz @ W4.T) * (1.0 - h3 ** 2)
    gW3, gb3 = h2.T @ d3, d3.sum(0)
    d2 = (d3 @ W3.T) * (1.0 - h2 ** 2)
    gW2, gb2 = h1.T @ d2, d2.sum(0)
    d1 = (d2 @ W2.T) * (1.0 - h1 ** 2)
    gW1, gb1 = X.T @ d1, d1.sum(0)
    return np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) with bias correction; step counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
