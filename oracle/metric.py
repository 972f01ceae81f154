"""Preparation of the three-index factors b from the metric (Sec. II, RI).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The four-centre integrals are approximated by (mu nu|k) G^-1 (l|sigma lambda)
with the metric G_kl = (k|l).  G may be ill conditioned, so it is factorised
symmetrically with pivoting, G = P L D L^T P^T, L unit lower triangular and D
block diagonal with 1x1 and 2x2 blocks (Bunch-Kaufman partial pivoting); the
eigenvalues of each D block below a threshold are raised to it (Cheng-Higham),
giving D~; then b solves  P L D~^(1/2) b^T = T,  T[k][mu nu] = (mu nu|k).  Every
b^k is symmetric in (mu, nu), and sum_k b^k_{mu nu} b^k_{sigma lambda} =
T^T G~^-1 T with G~ = P L D~ L^T P^T (= G when nothing is corrected).

Readings where the paper is silent:
  * The pivoting rule is the Bunch-Kaufman one with alpha = (1 + sqrt 17)/8,
    unblocked, on the lower triangle: at column k, with colmax the largest
    |G_ik| below the diagonal (row imax) and rowmax the largest off-diagonal
    |G_{imax,j}| of row imax in the trailing matrix: a 1x1 pivot at k if
    |G_kk| >= alpha colmax or |G_kk| rowmax >= alpha colmax^2; else a 1x1
    pivot at imax if |G_{imax,imax}| >= alpha rowmax; else a 2x2 pivot on
    (k, imax).  Ties in the column search go to the lowest index.  Interchanges
    are applied to the rows of the L columns already computed too, so the
    result is in the P L form.
  * Threshold of the correction: delta = sqrt(2^-52) * ||G||_inf (max row sum
    of |G|); eigenvalues of a D block below delta become delta.
  * perm: (P^T x)[i] = x[perm[i]].
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

__all__ = ["ALPHA", "bunch_kaufman", "correction_threshold", "corrected_blocks", "block_apply",
           "prepare_b", "reconstruct"]

ALPHA = (1.0 + np.sqrt(17.0)) / 8.0


def bunch_kaufman(G):
    """G = P L D L^T P^T.  Returns perm, L (unit lower), D (block diagonal,
    dense), and the block sizes (1 or 2, in order)."""
    A = np.array(G, dtype=np.float64)
    n = A.shape[0]
    L = np.eye(n)
    D = np.zeros((n, n))
    perm = np.arange(n)
    steps = []

    def swap(i, j):
        # symmetric interchange of rows/columns i and j of A (full matrix kept
        # symmetric), rows i and j of the L columns already final, and perm
        A[[i, j], :] = A[[j, i], :]
        A[:, [i, j]] = A[:, [j, i]]
        L[[i, j], :k] = L[[j, i], :k]
        perm[[i, j]] = perm[[j, i]]

    k = 0
    while k < n:
        absakk = abs(A[k, k])
        if k + 1 < n:
            col = np.abs(A[k + 1:, k])
            imax = k + 1 + int(np.argmax(col))
            colmax = col.max()
        else:
            imax, colmax = k, 0.0
        if max(absakk, colmax) == 0.0:
            kstep, kp = 1, k          # zero column: D_kk = 0, L column zero
        elif absakk >= ALPHA * colmax:
            kstep, kp = 1, k
        else:
            row = np.concatenate([np.abs(A[imax, k:imax]), np.abs(A[imax + 1:, imax])])
            rowmax = row.max()
            if absakk * rowmax >= ALPHA * colmax * colmax:
                kstep, kp = 1, k
            elif abs(A[imax, imax]) >= ALPHA * rowmax:
                kstep, kp = 1, imax
            else:
                kstep, kp = 2, imax
        kk = k + kstep - 1
        if kp != kk:
            swap(kk, kp)
        if kstep == 1:
            d = A[k, k]
            D[k, k] = d
            if d != 0.0:
                l = A[k + 1:, k] / d
                L[k + 1:, k] = l
                A[k + 1:, k + 1:] -= np.outer(l, A[k + 1:, k])
        else:
            E = A[k:k + 2, k:k + 2].copy()
            D[k:k + 2, k:k + 2] = E
            W = A[k + 2:, k:k + 2] @ np.linalg.inv(E)
            L[k + 2:, k:k + 2] = W
            A[k + 2:, k + 2:] -= W @ A[k + 2:, k:k + 2].T
        steps.append(kstep)
        k += kstep
    return perm, L, D, steps


def correction_threshold(G):
    return np.sqrt(2.0 ** -52) * np.max(np.sum(np.abs(G), axis=1))


def corrected_blocks(D, steps, delta):
    """D~ (eigenvalues of each block raised to delta), D~^(1/2) and D~^(-1/2)."""
    n = D.shape[0]
    Dt, Dh, Dih = np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
    k = 0
    for s in steps:
        blk = D[k:k + s, k:k + s]
        w, Q = np.linalg.eigh(blk)
        w = np.maximum(w, delta)
        Dt[k:k + s, k:k + s] = (Q * w) @ Q.T
        Dh[k:k + s, k:k + s] = (Q * np.sqrt(w)) @ Q.T
        Dih[k:k + s, k:k + s] = (Q / np.sqrt(w)) @ Q.T
        k += s
    return Dt, Dh, Dih


def block_apply(M, X):
    return M @ X


def prepare_b(T, G, delta=None):
    """b [n_aux][n_bf][n_bf] from T[k][mu][nu] = (mu nu|k) and the metric G."""
    n_aux = G.shape[0]
    n_bf = T.shape[1]
    perm, L, D, steps = bunch_kaufman(G)
    if delta is None:
        delta = correction_threshold(G)
    _, _, Dih = corrected_blocks(D, steps, delta)
    X = T.reshape(n_aux, n_bf * n_bf)[perm]                       # P^T T
    Y = solve_triangular(L, X, lower=True, unit_diagonal=True)   # L Y = P^T T
    bT = Dih @ Y                                                  # D~^(1/2) b^T = Y
    return bT.reshape(n_aux, n_bf, n_bf), dict(perm=perm, L=L, D=D, steps=steps, delta=delta)


def reconstruct(perm, L, Dt):
    """G~ = P L D~ L^T P^T."""
    n = L.shape[0]
    P = np.zeros((n, n))
    P[perm, np.arange(n)] = 1.0
    return P @ L @ Dt @ L.T @ P.T
