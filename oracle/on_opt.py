"""Occupation-number (ON) optimisation at fixed orbitals, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (Sec. II, occupancy optimisation) optimises the ONs for fixed
orbitals.  It expresses them through auxiliary variables gamma, so that the
bounds 0 <= n <= 1 and the pairing normalisation hold automatically and the
minimisation is unconstrained.  J and K are built once per outer iteration.
The parametrisation is not printed; the reading used here:

  strong orbital g:   n_g = (1 + cos^2 gamma_g) / 2          in [1/2, 1]
  weak orbitals of g: n_{w_k} = (1 - n_g) * w_k, hyperspherical weights
      w_1 = cos^2 b_1, w_k = prod_{j<k} sin^2 b_j * cos^2 b_k, w_last = prod sin^2 b_j
  variables per pair g: [gamma_g, b_1 .. b_{ncwo-1}], stored at g*ncwo + j.
  Weak orbitals of a pair are taken in ascending orbital index.
  Cold start: n_g = 0.98, equal weak ONs.

The energy is Eq. (2) (via pnof7_ri.energy) at fixed H_pp, J, K.
"""
from __future__ import annotations

import numpy as np

from . import pnof7_ri as ri

__all__ = ["weak_lists", "gamma_to_n", "cold_start", "energy_n", "grad_n", "dn_dgamma",
           "energy_gamma", "grad_gamma", "optimize", "n_to_gamma"]


def weak_lists(pair_of, n_pairs):
    W = len(pair_of)
    return [[p for p in range(n_pairs, W) if pair_of[p] == g] for g in range(n_pairs)]


def _weights(beta):
    """Hyperspherical weights from ncwo-1 angles (sum to 1)."""
    m = len(beta) + 1
    w = np.empty(m)
    s = 1.0
    for k in range(m - 1):
        w[k] = s * np.cos(beta[k]) ** 2
        s *= np.sin(beta[k]) ** 2
    w[m - 1] = s
    return w


def gamma_to_n(gamma, pair_of, n_pairs, n_cwo):
    W = len(pair_of)
    n = np.zeros(W)
    weak = weak_lists(pair_of, n_pairs)
    for g in range(n_pairs):
        x = gamma[g * n_cwo: (g + 1) * n_cwo]
        n[g] = 0.5 * (1.0 + np.cos(x[0]) ** 2)
        w = _weights(x[1:])
        for k, p in enumerate(weak[g]):
            n[p] = (1.0 - n[g]) * w[k]
    return n


def n_to_gamma(n, pair_of, n_pairs, n_cwo):
    """Inverse map (angles in [0, pi/2])."""
    gamma = np.zeros(n_pairs * n_cwo)
    weak = weak_lists(pair_of, n_pairs)
    for g in range(n_pairs):
        c2 = min(max(2.0 * n[g] - 1.0, 0.0), 1.0)
        gamma[g * n_cwo] = np.arccos(np.sqrt(c2))
        h = max(1.0 - n[g], 1e-300)
        w = np.array([n[p] / h for p in weak[g]])
        s = 1.0
        for k in range(n_cwo - 1):
            c2 = min(max(w[k] / s, 0.0), 1.0) if s > 0 else 1.0
            gamma[g * n_cwo + 1 + k] = np.arccos(np.sqrt(c2))
            s *= 1.0 - c2
    return gamma


def cold_start(n_pairs, n_cwo, n_strong=0.98):
    gamma = np.zeros(n_pairs * n_cwo)
    for g in range(n_pairs):
        gamma[g * n_cwo] = np.arccos(np.sqrt(2.0 * n_strong - 1.0))
        for k in range(1, n_cwo):
            gamma[g * n_cwo + k] = np.arccos(np.sqrt(1.0 / (n_cwo - k + 1)))
    return gamma


def energy_n(n, Hpp, J, K, pair_of, n_pairs, functional="pnof7"):
    Delta, Pi = ri.delta_pi(n, pair_of, n_pairs, functional)
    return ri.energy(n, Hpp, J, K, Delta, Pi)


def grad_n(n, Hpp, J, K, pair_of, n_pairs, functional="pnof7"):
    """dE/dn_p of Eq. (2) with the PNOF7 reading, differentiated term by term."""
    W = len(n)
    phi = np.sqrt(n * (1.0 - n))
    dphi = (1.0 - 2.0 * n) / (2.0 * np.maximum(phi, 1e-300))
    g = 2.0 * Hpp.copy()
    for p in range(W):
        g[p] += K[p, p]                       # d(n_p K_pp)/dn_p (diagonal Pi_pp = n_p)
        for q in range(W):
            if q == p:
                continue
            if pair_of[p] == pair_of[q]:
                sgn = 1.0 if (p >= n_pairs and q >= n_pairs) else -1.0
                dB = sgn * 0.5 * np.sqrt(n[q] / max(n[p], 1e-300))
                g[p] += 2.0 * dB * K[p, q]
            else:
                dA = 2.0 * n[q]
                dB = -n[q] - (dphi[p] * phi[q] if functional == "pnof7" else 0.0)
                g[p] += 2.0 * (dA * J[p, q] + dB * K[p, q])
    return g


def dn_dgamma(gamma, pair_of, n_pairs, n_cwo):
    """Jacobian dn/dgamma ([W][n_pairs*n_cwo]) by the chain rule of the map."""
    W = len(pair_of)
    D = np.zeros((W, n_pairs * n_cwo))
    weak = weak_lists(pair_of, n_pairs)
    for g in range(n_pairs):
        x = gamma[g * n_cwo: (g + 1) * n_cwo]
        c, s = np.cos(x[0]), np.sin(x[0])
        D[g, g * n_cwo] = -c * s                         # d n_g / d gamma_g
        h = 0.5 * s * s
        dh = c * s
        beta = x[1:]
        w = _weights(beta)
        m = n_cwo
        # dw_k / dbeta_j
        dw = np.zeros((m, m - 1))
        for k in range(m):
            for j in range(m - 1):
                if j > k or (j == k and k == m - 1):
                    continue
                val = 1.0
                for i in range(min(k, m - 1)):
                    val *= (2 * np.sin(beta[i]) * np.cos(beta[i])) if i == j else np.sin(beta[i]) ** 2
                if k < m - 1:
                    val *= (-2 * np.cos(beta[k]) * np.sin(beta[k])) if j == k else np.cos(beta[k]) ** 2
                dw[k, j] = val
        for k, p in enumerate(weak[g]):
            D[p, g * n_cwo] = dh * w[k]
            for j in range(m - 1):
                D[p, g * n_cwo + 1 + j] = h * dw[k, j]
    return D


def energy_gamma(gamma, Hpp, J, K, pair_of, n_pairs, n_cwo, functional="pnof7"):
    return energy_n(gamma_to_n(gamma, pair_of, n_pairs, n_cwo), Hpp, J, K, pair_of, n_pairs, functional)


def grad_gamma(gamma, Hpp, J, K, pair_of, n_pairs, n_cwo, functional="pnof7"):
    n = gamma_to_n(gamma, pair_of, n_pairs, n_cwo)
    return dn_dgamma(gamma, pair_of, n_pairs, n_cwo).T @ grad_n(n, Hpp, J, K, pair_of, n_pairs, functional)


def optimize(Hpp, J, K, pair_of, n_pairs, n_cwo, gamma0=None, tol=1e-8, max_it=2000,
             functional="pnof7"):
    """Reference minimiser (scipy L-BFGS-B without bounds) to max|dE/dgamma| <= tol."""
    from scipy.optimize import minimize
    x0 = cold_start(n_pairs, n_cwo) if gamma0 is None else np.asarray(gamma0, dtype=float)
    f = lambda x: energy_gamma(x, Hpp, J, K, pair_of, n_pairs, n_cwo, functional)
    gf = lambda x: grad_gamma(x, Hpp, J, K, pair_of, n_pairs, n_cwo, functional)
    res = minimize(f, x0, jac=gf, method="L-BFGS-B",
                   options={"maxiter": max_it, "gtol": tol, "ftol": 0.0, "maxcor": 10})
    return res.x, res.fun, res.nit, float(np.max(np.abs(gf(res.x))))
