"""Learned warm start for the occupation-number (ON) optimisation.

The occupancy optimisation (Sec. II) is cheap once J and K exist, but it is
iterative.  A small MLP, trained on data the method itself generates
(converged ONs of many molecules), predicts each pair's ONs from per-pair
features of H_pp, J and K.  The prediction becomes the starting point of the
plain ON optimiser, which still decides the result: it iterates to
max|dE/dgamma| <= tol from wherever it starts.

Every numerical step runs in librif kernels (J/K, H_pp, features, MLP
forward/backward, Adam, ON optimiser); this module only sequences the calls
and holds device buffers.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import FP64, PNOF7, Context, OnSet

N_IN, N_HID, N_OUT = 39, 128, 7


def jk_problem(ctx: Context, inp, n_pairs, n_cwo, prec=FP64):
    """J, K (Table 2 steps 2-4) and H_pp of one molecule on the GPU."""
    w = n_pairs * (1 + n_cwo)
    bh, bmo, d = ctx.transform(inp["b"], inp["C"], w, prec)
    J, K = ctx.jk_mo(bmo, d, prec)
    Hpp = ctx.hpp(inp["H"], inp["C"], w)
    del bh, bmo, d
    return (Hpp, J, K, inp.get("pair_of"), n_pairs, n_cwo)


def prior_rows(onset: OnSet, n_strong=0.98):
    """Cold-start ONs (strong 0.98, weak equal) as prediction rows [rows][7]."""
    import torch
    P = torch.zeros((onset.rows, N_OUT), dtype=torch.float32)
    r = 0
    for npair, ncwo in onset.sizes:
        P[r:r + npair, 0] = n_strong
        P[r:r + npair, 1:1 + min(ncwo, 6)] = (1.0 - n_strong) / ncwo
        r += npair
    return P.to(onset.gamma.device)


class WarmStartMLP:
    """39 -> 128 -> 128 -> 128 -> 7 network on the GPU (FP32)."""

    def __init__(self, ctx: Context, seed=0, device="cuda"):
        import torch
        self.ctx = ctx
        self.device = device
        n = ctx.mlp_n_params()
        rng = np.random.default_rng(seed)
        parts = []
        for i, o in ((N_IN, N_HID), (N_HID, N_HID), (N_HID, N_HID), (N_HID, N_OUT)):
            a = math.sqrt(6.0 / (i + o))
            parts += [rng.uniform(-a, a, size=i * o), np.zeros(o)]
        theta = np.concatenate(parts)
        assert theta.size == n
        self.theta = torch.from_numpy(theta.astype(np.float32)).to(device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.step = 0
        self.mu = None
        self.sigma = None

    def _bufs(self, rows):
        import torch
        f = torch.float32
        return (torch.empty((3, rows, N_HID), dtype=f, device=self.device),
                torch.empty((rows, N_OUT), dtype=f, device=self.device),
                torch.empty((rows, N_OUT), dtype=f, device=self.device))

    def fit(self, X, T, M, epochs=400, lr=3e-3, lr_final=None):
        """Full-batch Adam on the GPU, the learning rate decaying geometrically
        from lr to lr_final (default: constant); returns the loss history."""
        import torch
        rows = X.shape[0]
        H, Z, P = self._bufs(rows)
        dA = torch.empty((2, rows, N_HID), dtype=torch.float32, device=self.device)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        hist = []
        decay = 1.0 if lr_final is None else (lr_final / lr) ** (1.0 / max(1, epochs - 1))
        for e in range(epochs):
            self.ctx.mlp_forward(X, M, self.theta, H, Z, P)
            self.ctx.mlp_backward(X, M, T, self.theta, H, Z, dA, self.grad, loss)
            self.step += 1
            self.ctx.adam(self.theta, self.grad, self.m, self.v, self.step, lr * decay ** e)
            hist.append(loss)
            loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        return [float(h.item()) for h in hist]

    def predict(self, X, M):
        H, Z, P = self._bufs(X.shape[0])
        self.ctx.mlp_forward(X, M, self.theta, H, Z, P)
        return P

    def save(self, path, mu=None, sigma=None):
        """The weights, the Adam state and the feature standardisation (mu,
        sigma; defaults: the ones set on the network) to an .npz file of
        plain arrays, so a trained warm start can be reused without training."""
        mu = self.mu if mu is None else mu
        sigma = self.sigma if sigma is None else sigma
        arrs = {"layers": np.array([N_IN, N_HID, N_HID, N_HID, N_OUT], dtype=np.int64),
                "theta": self.theta.detach().cpu().numpy(), "m": self.m.detach().cpu().numpy(),
                "v": self.v.detach().cpu().numpy(), "step": np.array([self.step], dtype=np.int64)}
        for k, x in (("mu", mu), ("sigma", sigma)):
            if x is not None:
                arrs[k] = (x.detach().cpu().numpy() if hasattr(x, "detach") else np.asarray(x)).astype(np.float32)
        np.savez(path, **arrs)

    @classmethod
    def load(cls, ctx: Context, path, device="cuda"):
        """A network written by save(); mu and sigma come back as attributes
        (None if they were not saved).  Raises ValueError for another layout."""
        import torch
        with np.load(path, allow_pickle=False) as f:
            missing = [k for k in ("layers", "theta", "m", "v", "step") if k not in f]
            if missing:
                raise ValueError(f"{path}: no {', '.join(missing)}")
            if not np.array_equal(f["layers"], [N_IN, N_HID, N_HID, N_HID, N_OUT]):
                raise ValueError(f"{path}: layer sizes {f['layers'].tolist()} differ from this network's")
            net = cls(ctx, device=device)
            n = ctx.mlp_n_params()
            for k in ("theta", "m", "v"):
                a = f[k]
                if a.shape != (n,):
                    raise ValueError(f"{path}: {k} has shape {a.shape}, expected ({n},)")
                setattr(net, k, torch.from_numpy(a.astype(np.float32)).to(device))
            net.step = int(f["step"][0])
            for k in ("mu", "sigma"):
                if k in f:
                    a = f[k]
                    if a.shape != (N_IN,):
                        raise ValueError(f"{path}: {k} has shape {a.shape}, expected ({N_IN},)")
                    setattr(net, k, torch.from_numpy(a.astype(np.float32)).to(device))
        return net


def features(ctx: Context, onset: OnSet, with_targets=False, mu=None, sigma=None):
    import torch
    f = torch.float32
    dev = onset.gamma.device
    X = torch.empty((onset.rows, N_IN), dtype=f, device=dev)
    M = torch.empty((onset.rows, N_OUT), dtype=f, device=dev)
    T = torch.empty((onset.rows, N_OUT), dtype=f, device=dev) if with_targets else None
    ctx.on_features(onset, X, T, M, mu, sigma)
    return X, T, M


def standardisation(X):
    """Per-feature mean and spread of the training features (host statistics)."""
    import torch
    x = X.detach().cpu().double().numpy()
    mu = x.mean(0)
    sd = x.std(0)
    sd[sd < 1e-12] = 0.0           # constant columns (the slot masks) pass through
    mu[sd == 0.0] = 0.0
    return (torch.from_numpy(mu.astype(np.float32)).to(X.device),
            torch.from_numpy(sd.astype(np.float32)).to(X.device))


def solve(ctx: Context, onset: OnSet, P):
    """Start every problem from predicted ONs P and run the plain optimiser.
    Returns (iterations per problem, status per problem, seconds of GPU time)."""
    import torch
    ctx.on_warmstart(onset, P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.on_optimize(onset)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return onset.iters.cpu().numpy().copy(), onset.status.cpu().numpy().copy(), dt
