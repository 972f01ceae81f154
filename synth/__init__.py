"""Seeded synthetic inputs for the RI-PNOF7 hot path.

This module draws random numbers and lays them out; it holds none of the
method's arithmetic (no transform, no J/K build, no energy).  Both the HIP
path (through the binding) and the CPU oracle consume what it returns.

Workloads (shapes mimic the paper's cc-pVTZ-class molecules; the paper's own
molecules, basis sets and integrals are not available, so these synthetic
inputs stand in for them):

  name     n_bf  n_aux  pairs  ncwo  n_omega  n_mo
  tiny       48    192      5     1       10    48   (oracle-sized)
  c6h12     348   1044     24     4      120   348   (cyclohexane-like)
  c10h20    580   1740     40     4      200   580   (cyclodecane-like)
  batch64   U{60..400}, 3*n_bf, n_bf//12, 2          (64 uneven molecules)
  large    1000   3000     60     6      420  1000

Recipe (draw order b -> C -> H -> ON, numpy ``default_rng(seed)``):
  b[P] = (G_P + G_P^T)/2 * exp(-3P/n_aux),  G_P ~ N(0, 1/n_bf) i.i.d.
  C    = Q of the QR factorisation of an n_bf x n_mo standard-normal matrix
  H    = symmetric: upper triangle N(0,1), mirrored
  ON   : per pair, strong ON ~ U(0.9, 0.99); each of the ncwo weak orbitals
         of the pair gets (1 - strong)/ncwo, so every pair sums to exactly 1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Instance", "WORKLOADS", "default_pair_map", "make_instance", "make_b",
    "rotation_sequence", "batch_sizes", "make_batch", "make_batch_device", "make_instance_device",
    "make_metric", "make_three_centre",
]

# name -> (n_bf, n_aux, n_pairs, n_cwo, seed)
WORKLOADS = {
    "tiny": (48, 192, 5, 1, 0),
    "c6h12": (348, 1044, 24, 4, 1),
    "c10h20": (580, 1740, 40, 4, 2),
    "large": (1000, 3000, 60, 6, 4),
}


@dataclasses.dataclass
class Instance:
    """One molecule's worth of inputs.  All arrays are C-ordered float64/int32."""
    n_bf: int
    n_aux: int
    n_pairs: int
    n_cwo: int
    n_mo: int
    b: np.ndarray        # [n_aux][n_bf][n_bf], each slab symmetric
    C: np.ndarray        # [n_bf][n_mo], orthonormal columns
    H: np.ndarray        # [n_bf][n_bf], symmetric
    occ: np.ndarray      # [n_omega]
    pair_of: np.ndarray  # [n_omega] int32: pair index of each orbital in Omega
    seed: int = 0

    @property
    def n_omega(self) -> int:
        return self.n_pairs * (1 + self.n_cwo)


def default_pair_map(n_pairs: int, n_cwo: int) -> np.ndarray:
    """Orbital -> pair map of the electron-pairing scheme.

    Orbitals 0..n_pairs-1 are the strong (doubly occupied in the HF limit)
    orbitals; orbital g is the strong orbital of pair g.  The weak orbitals
    of pair g are n_pairs + n_cwo*(n_pairs-1-g) + k, k = 0..n_cwo-1, so the
    highest strong orbital couples to the lowest weak ones.
    """
    W = n_pairs * (1 + n_cwo)
    pm = np.empty(W, dtype=np.int32)
    pm[:n_pairs] = np.arange(n_pairs)
    for g in range(n_pairs):
        for k in range(n_cwo):
            pm[n_pairs + n_cwo * (n_pairs - 1 - g) + k] = g
    return pm


def make_b(rng: np.random.Generator, n_bf: int, n_aux: int, out=None) -> np.ndarray:
    """Three-index factors, drawn slab by slab to bound host memory."""
    b = np.empty((n_aux, n_bf, n_bf), dtype=np.float64) if out is None else out
    s = 1.0 / math.sqrt(n_bf)
    for P in range(n_aux):
        G = rng.standard_normal((n_bf, n_bf))
        G *= s
        np.add(G, G.T, out=b[P])
        b[P] *= 0.5 * math.exp(-3.0 * P / n_aux)
    return b


def make_instance(n_bf: int, n_aux: int, n_pairs: int, n_cwo: int, seed: int,
                  n_mo: int | None = None, strong_range=(0.9, 0.99)) -> Instance:
    n_mo = n_bf if n_mo is None else n_mo
    W = n_pairs * (1 + n_cwo)
    if W > n_mo or n_mo > n_bf:
        raise ValueError("need n_omega <= n_mo <= n_bf")
    rng = np.random.default_rng(seed)
    b = make_b(rng, n_bf, n_aux)
    X = rng.standard_normal((n_bf, n_mo))
    C, _ = np.linalg.qr(X)
    C = np.ascontiguousarray(C)
    Hx = rng.standard_normal((n_bf, n_bf))
    H = np.triu(Hx) + np.triu(Hx, 1).T
    strong = rng.uniform(strong_range[0], strong_range[1], size=n_pairs)
    pair_of = default_pair_map(n_pairs, n_cwo)
    occ = np.empty(W, dtype=np.float64)
    occ[:n_pairs] = strong
    for i in range(n_pairs, W):
        occ[i] = (1.0 - strong[pair_of[i]]) / n_cwo
    return Instance(n_bf, n_aux, n_pairs, n_cwo, n_mo, b, C, np.ascontiguousarray(H),
                    occ, pair_of, seed)


def workload(name: str) -> Instance:
    n_bf, n_aux, n_pairs, n_cwo, seed = WORKLOADS[name]
    return make_instance(n_bf, n_aux, n_pairs, n_cwo, seed)


def rotation_sequence(C0: np.ndarray, n_iter: int, base_seed: int = 1000,
                      scale: float = 0.01) -> list:
    """Orbitals of a fixed-rotation sequence: C_{it+1} = C_it expm(kappa_it),
    kappa_it = scale*(X - X^T)/2 with X ~ N(0,1) from seed base_seed+it.
    Returns [C_0, C_1, ..., C_{n_iter-1}] (C_0 is the input)."""
    from scipy.linalg import expm
    n = C0.shape[1]
    out = [np.ascontiguousarray(C0)]
    C = C0
    for it in range(n_iter - 1):
        X = np.random.default_rng(base_seed + it).standard_normal((n, n))
        kappa = scale * 0.5 * (X - X.T)
        C = np.ascontiguousarray(C @ expm(kappa))
        out.append(C)
    return out


def batch_sizes(n_inst: int = 64, seed: int = 3, lo: int = 60, hi: int = 400) -> np.ndarray:
    """n_bf of each molecule of the uneven batch, uniform on {lo..hi}."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=n_inst)


def make_batch(n_inst: int = 64, seed: int = 3, base: int = 3000, n_cwo: int = 2,
               lo: int = 60, hi: int = 400) -> list:
    """Uneven batch: n_aux = 3 n_bf, pairs = n_bf // 12, per-instance seed base+i."""
    return [make_instance(int(nb), 3 * int(nb), int(nb) // 12, n_cwo, base + i)
            for i, nb in enumerate(batch_sizes(n_inst, seed, lo, hi))]


def make_instance_device(n_bf: int, n_aux: int, n_pairs: int, n_cwo: int, seed: int, device="cuda",
                         n_mo: int | None = None):
    """Same recipe as make_instance, with b drawn on the GPU (torch.Generator
    seeded with `seed`) so that large or many instances are cheap to make; C, H
    and the ONs come from numpy default_rng(seed + 2**32) in the order C -> H -> ON.
    The streams differ from make_instance's, so the two never mix in one test.
    Returns (dict of device tensors b, C, H, occ, pair_of; n_pairs; n_cwo)."""
    import torch
    n_mo = n_bf if n_mo is None else n_mo
    W = n_pairs * (1 + n_cwo)
    if W > n_mo or n_mo > n_bf:
        raise ValueError("need n_omega <= n_mo <= n_bf")
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    b = torch.empty((n_aux, n_bf, n_bf), dtype=torch.float64, device=device)
    scale = torch.exp(-3.0 * torch.arange(n_aux, dtype=torch.float64, device=device) / n_aux)
    chunk = max(1, (1 << 27) // (n_bf * n_bf))
    for p0 in range(0, n_aux, chunk):
        p1 = min(n_aux, p0 + chunk)
        G = torch.randn((p1 - p0, n_bf, n_bf), dtype=torch.float64, device=device, generator=gen)
        G *= 1.0 / math.sqrt(n_bf)
        b[p0:p1] = (G + G.transpose(1, 2)) * (0.5 * scale[p0:p1, None, None])
        del G
    rng = np.random.default_rng(seed + 2 ** 32)
    C, _ = np.linalg.qr(rng.standard_normal((n_bf, n_mo)))
    Hx = rng.standard_normal((n_bf, n_bf))
    H = np.triu(Hx) + np.triu(Hx, 1).T
    strong = rng.uniform(0.9, 0.99, size=n_pairs)
    pair_of = default_pair_map(n_pairs, n_cwo)
    occ = np.empty(W)
    occ[:n_pairs] = strong
    for i in range(n_pairs, W):
        occ[i] = (1.0 - strong[pair_of[i]]) / n_cwo
    t = {"b": b, "C": torch.from_numpy(np.ascontiguousarray(C)).to(device),
         "H": torch.from_numpy(np.ascontiguousarray(H)).to(device), "occ": torch.from_numpy(occ).to(device),
         "pair_of": torch.from_numpy(pair_of.astype(np.int32)).to(device)}
    return t, n_pairs, n_cwo


def make_batch_device(n_inst: int = 64, seed: int = 3, base: int = 3000, n_cwo: int = 2,
                      lo: int = 60, hi: int = 400, device="cuda") -> list:
    """The uneven batch with b drawn on the GPU (make_instance_device, seed
    base+i): n_bf ~ U{lo..hi} (batch_sizes), n_aux = 3 n_bf, pairs = n_bf // 12.
    Returns a list of (dict of device tensors, n_pairs, n_cwo)."""
    return [make_instance_device(int(nb), 3 * int(nb), int(nb) // 12, n_cwo, base + i, device=device)
            for i, nb in enumerate(batch_sizes(n_inst, seed, lo, hi))]


def make_metric(n_aux: int, seed: int, cond: float = 1e10, n_negative: int = 0) -> np.ndarray:
    """Symmetric metric stand-in G = Q diag(w) Q^T, Q from the QR of a seeded
    Gaussian matrix, w geometric from 1 down to 1/cond; the last n_negative
    eigenvalues are replaced by -1e-3/cond (a numerically indefinite metric,
    as real auxiliary-basis metrics can be)."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n_aux, n_aux)))
    w = np.geomspace(1.0, 1.0 / cond, n_aux)
    if n_negative:
        w[-n_negative:] = -1e-3 / cond
    G = (Q * w) @ Q.T
    return (G + G.T) / 2


def make_three_centre(n_bf: int, n_aux: int, seed: int) -> np.ndarray:
    """T[k][mu][nu] = (mu nu|k) stand-in: symmetric Gaussian slabs
    (X + X^T)/2, X ~ N(0, 1/n_bf)."""
    rng = np.random.default_rng(seed)
    T = np.empty((n_aux, n_bf, n_bf))
    for k in range(n_aux):
        X = rng.standard_normal((n_bf, n_bf)) / np.sqrt(n_bf)
        T[k] = (X + X.T) / 2
    return T

