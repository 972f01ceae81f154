"""Orbital optimisation by iterative diagonalisation, and the outer/inner loop.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. II, orbital optimisation with RI: for fixed ONs the natural orbitals are
found by diagonalising, again and again, a symmetric matrix F^lambda made from
the Lagrange multipliers of the orthonormality constraints; the eigenvectors
rotate the orbitals, so orthonormality holds at every step.  The diagonal of
F^lambda is not fixed by lambda and is set by an aufbau rule.  The general
scheme (Fig. 1) alternates an ON optimisation at fixed orbitals (outer
iteration) with many such orbital steps at fixed ONs (inner iterations).

The paper does not print F^lambda; the reading used here (from the iterative
diagonalisation work it cites):
  * lambda_ab = c_a^T F^(b) c_b as in pnof7_ri.lagrangian, zero for b outside
    Omega, extended to an n_mo x n_mo matrix.
  * Off-diagonal: F_pq = lambda_{hi,lo} - lambda_{lo,hi} with hi = max(p, q),
    lo = min(p, q).  F is symmetric and vanishes off the diagonal exactly when
    lambda is symmetric, i.e. when the orbital gradient G = 4 (lambda - lambda^T)
    is zero.
  * Diagonal (aufbau): lambda_pp at the first step of an inner loop, then the
    eigenvalues of the previous step.  Eigenvectors are taken in ascending
    eigenvalue order, so orbital p of the new set is the p-th lowest; its role
    (strong or weak orbital of a pair, or outside Omega) follows its index.
  * With ascending diagonal values this makes every small step a descent step:
    to first order the rotation is kappa_qp = F_qp / (eps_p - eps_q) and the
    energy change is -4 sum_{q<p} (lambda_qp - lambda_pq)^2 / (eps_p - eps_q).
  * Outer loop: ON optimisation (on_opt.optimize, started from the previous
    gamma) at the current orbitals, then inner iterations at the new ONs until
    max|G| <= tol_grad; converged once an outer iteration changes the energy
    by at most tol_energy and its inner loop converged.
"""
from __future__ import annotations

import numpy as np

from . import on_opt
from . import pnof7_ri as ri

__all__ = ["lambda_full", "fock_lambda", "orbital_step", "inner_loop", "outer_loop"]


def lambda_full(lam: np.ndarray, n_mo: int) -> np.ndarray:
    """[n_mo][n_omega] multipliers -> [n_mo][n_mo], zero columns outside Omega."""
    full = np.zeros((n_mo, n_mo))
    full[:, :lam.shape[1]] = lam
    return full


def fock_lambda(lam: np.ndarray, n_mo: int, eps=None) -> np.ndarray:
    """F^lambda of the orbital step (reading above)."""
    L = lambda_full(lam, n_mo)
    lower = np.tril(L - L.T, -1)          # entry (hi, lo): lambda_hi,lo - lambda_lo,hi
    F = lower + lower.T
    F[np.diag_indices(n_mo)] = np.diag(L) if eps is None else eps
    return F


def orbital_step(C: np.ndarray, lam: np.ndarray, eps=None):
    """One diagonalisation: returns (C V, eigenvalues ascending)."""
    F = fock_lambda(lam, C.shape[1], eps)
    w, V = np.linalg.eigh(F)
    return C @ V, w


def inner_loop(b, C, H, occ, pair_of, n_pairs, max_it, tol_grad, functional="pnof7"):
    """Inner iterations at fixed ONs.  Each iteration is one build (energy,
    lambda, G at the current orbitals); if max|G| <= tol_grad the loop stops,
    otherwise one orbital step follows.  Returns the final orbitals, the last
    eigenvalues, and per-iteration energies and max|G|."""
    energies, grads = [], []
    eps = None
    converged = False
    for _ in range(max_it):
        r = ri.build(b, C, H, occ, pair_of, n_pairs, functional)
        energies.append(r["energy"])
        grads.append(float(np.max(np.abs(r["grad"]))))
        if grads[-1] <= tol_grad:
            converged = True
            break
        C, eps = orbital_step(C, r["lam"], eps)
    return dict(C=C, eps=eps, energies=energies, grads=grads, converged=converged)


def outer_loop(b, C, H, occ, pair_of, n_pairs, n_cwo, max_outer, max_inner, tol_grad,
               tol_energy, on_tol=1e-10, functional="pnof7"):
    """Fig. 1: alternate ON optimisation (fixed orbitals) and orbital
    optimisation (fixed ONs).  Returns orbitals, ONs, gamma, energy history
    (one entry per outer iteration: the energy at the end of its inner loop),
    the inner iteration counts and whether the loop converged."""
    W = occ.shape[0]
    gamma = on_opt.n_to_gamma(occ, pair_of, n_pairs, n_cwo)
    energies, inner_counts = [], []
    converged = False
    for _ in range(max_outer):
        Co = np.ascontiguousarray(C[:, :W])
        bh = ri.half_transform(b, Co)
        J, K = ri.jk_mo(ri.mo_transform(bh, Co))
        Hp = ri.hpp(H, Co)
        gamma, _, _, _ = on_opt.optimize(Hp, J, K, pair_of, n_pairs, n_cwo, gamma0=gamma,
                                         tol=on_tol, functional=functional)
        occ = on_opt.gamma_to_n(gamma, pair_of, n_pairs, n_cwo)
        res = inner_loop(b, C, H, occ, pair_of, n_pairs, max_inner, tol_grad, functional)
        C = res["C"]
        inner_counts.append(len(res["energies"]))
        energies.append(res["energies"][-1])
        if (res["converged"] and len(energies) > 1
                and abs(energies[-1] - energies[-2]) <= tol_energy):
            converged = True
            break
    return dict(C=C, occ=occ, gamma=gamma, energies=energies, inner=inner_counts,
                converged=converged)
