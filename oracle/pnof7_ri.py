"""Plain FP64 definition of the RI-PNOF7 per-iteration hot path.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function is the
textbook definition of one step, written with numpy library primitives
(matmul, einsum) and no blocking, fusion or reordering beyond what the
definition states.

Index names: l = auxiliary index (0..n_aux-1), mu/nu = AO index
(0..n_bf-1), p/q/r = orbitals of the pairing scheme Omega (0..n_omega-1),
a = any MO (0..n_mo-1).  Omega is the first n_omega columns of C.

Readings where the paper is silent (each also listed in the design notes):
  * The PNOF7 Delta and Pi matrices are not written out in the paper (only
    the generic form of Eq. (2)); they are taken from the PNOF7 functional the
    paper cites:  within a pair subspace Delta_qp = n_q n_p and
    Pi_qp = +sqrt(n_q n_p) if both orbitals are weak, -sqrt(n_q n_p) if one
    is the strong orbital, Pi_pp = n_p;  between pairs Delta_qp = 0 and
    Pi_qp = -Phi_q Phi_p with Phi_p = sqrt(n_p (1-n_p)) (PNOF7; PNOF5 drops
    this term).
  * The strong orbital of pair g is orbital g (g < n_pairs).
  * The Lagrangian is lambda_ab = c_a^T F^(b) c_b with
    F^(b) = n_b H + sum_r (A_br J^(r) + B_br K^(r)), zero for b outside
    Omega, and the orbital gradient is G = 4 (lambda - lambda^T); G_ab is the
    derivative of E along C -> C expm(theta (E_ab - E_ba)).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "half_transform", "mo_transform", "diag_of", "jk_mo", "jk_ao_per_mo",
    "delta_pi", "coefficients", "hpp", "energy", "energy_from_coefficients",
    "lagrangian", "lagrangian_direct", "build",
]


def half_transform(b: np.ndarray, C_omega: np.ndarray) -> np.ndarray:
    """Eq. (12); Table 2 step 2 and Table 3 step 2.

    b_half[p][l][nu] = sum_mu C[mu][p] b[l][mu][nu]   ->  [n_omega][n_aux][n_bf]
    """
    # matmul over the leading l axis: (C^T)[p][mu] b[l][mu][nu]
    t = np.matmul(C_omega.T[None, :, :], b)          # [l][p][nu]
    return np.ascontiguousarray(t.transpose(1, 0, 2))


def mo_transform(b_half: np.ndarray, C_omega: np.ndarray) -> np.ndarray:
    """Eq. (13); Table 2 step 3.

    b_mo[l][p][q] = sum_nu C[nu][q] b_half[p][l][nu]   ->  [n_aux][n_omega][n_omega]
    """
    t = np.matmul(b_half, C_omega[None, :, :])          # [p][l][q]
    return np.ascontiguousarray(t.transpose(1, 0, 2))


def diag_of(b_mo: np.ndarray) -> np.ndarray:
    """d[l][q] = b^l_qq (Table 3 step 3, Coulomb branch)."""
    return np.ascontiguousarray(np.diagonal(b_mo, axis1=1, axis2=2))


def jk_mo(b_mo: np.ndarray):
    """Eqs. (10)-(11); Table 2 step 4.

    J[p][q] = sum_l b^l_pp b^l_qq,   K[p][q] = sum_l (b^l_pq)^2
    """
    d = diag_of(b_mo)
    J = d.T @ d
    K = np.einsum("lpq,lpq->pq", b_mo, b_mo)
    return J, K


def jk_ao_per_mo(b: np.ndarray, b_half: np.ndarray, d: np.ndarray):
    """Table 3 steps 3-4.

    Jn[q][mu][nu] = sum_l b^l_qq b^l_{mu nu}
    Kn[q][mu][nu] = sum_l b^l_{q mu} b^l_{q nu}
    """
    A, B, _ = b.shape
    W = d.shape[1]
    Jn = (d.T @ b.reshape(A, B * B)).reshape(W, B, B)
    Kn = np.matmul(b_half.transpose(0, 2, 1), b_half)   # [q][mu][l] @ [q][l][nu]
    return Jn, Kn


def delta_pi(occ: np.ndarray, pair_of: np.ndarray, n_pairs: int,
             functional: str = "pnof7"):
    """Delta and Pi of Eq. (2) for the electron-pairing PNOFs (reading above)."""
    W = occ.shape[0]
    phi = np.sqrt(occ * (1.0 - occ))
    Delta = np.zeros((W, W))
    Pi = np.zeros((W, W))
    for q in range(W):
        for p in range(W):
            if pair_of[q] == pair_of[p]:
                Delta[q, p] = occ[q] * occ[p]
                if q == p:
                    Pi[q, p] = occ[p]
                elif q >= n_pairs and p >= n_pairs:
                    Pi[q, p] = np.sqrt(occ[q] * occ[p])
                else:
                    Pi[q, p] = -np.sqrt(occ[q] * occ[p])
            else:
                Delta[q, p] = 0.0
                Pi[q, p] = -phi[q] * phi[p] if functional == "pnof7" else 0.0
    return Delta, Pi


def coefficients(occ, pair_of, n_pairs, functional="pnof7"):
    """Eq. (2) with L = K, regrouped as E = 2 sum n_p H_pp + sum_pq (A_pq J_pq + B_pq K_pq):
    A_pq = 2 (n_q n_p - Delta_qp),  B_pq = Pi_qp - (n_q n_p - Delta_qp)."""
    Delta, Pi = delta_pi(occ, pair_of, n_pairs, functional)
    X = np.outer(occ, occ) - Delta
    return 2.0 * X.T, (Pi - X).T


def hpp(H: np.ndarray, C_omega: np.ndarray) -> np.ndarray:
    """H_pp = c_p^T H c_p (Eq. (1), one-electron part)."""
    return np.einsum("mp,mn,np->p", C_omega, H, C_omega)


def energy(occ, Hpp, J, K, Delta, Pi) -> float:
    """Eq. (2) term by term, with L_pq = K_pq for real orbitals."""
    nn = np.outer(occ, occ)
    E = 2.0 * np.sum(occ * Hpp)
    E += np.sum(Pi * K.T)                       # sum_qp Pi_qp L_pq
    E += np.sum((nn - Delta) * (2.0 * J.T - K.T))
    return float(E)


def energy_from_coefficients(occ, Hpp, J, K, A, B) -> float:
    return float(2.0 * np.sum(occ * Hpp) + np.sum(A * J) + np.sum(B * K))


def lagrangian(H, C, occ, Jn, Kn, A, B):
    """Lagrange multipliers and orbital gradient (the orbital-optimisation
    quantities the paper says are needed every inner iteration).

    F^(q) = n_q H + sum_r (A_qr J^(r) + B_qr K^(r));  Y[:, q] = F^(q) c_q;
    lambda = C^T Y  ([n_mo][n_omega], columns outside Omega are zero);
    G = 4 (lambda - lambda^T)  ([n_mo][n_mo]).
    """
    W, B_, _ = Jn.shape
    n_mo = C.shape[1]
    FJ = (A @ Jn.reshape(W, B_ * B_)).reshape(W, B_, B_)
    FK = (B @ Kn.reshape(W, B_ * B_)).reshape(W, B_, B_)
    Y = np.empty((B_, W))
    for q in range(W):
        F = occ[q] * H + FJ[q] + FK[q]
        Y[:, q] = F @ C[:, q]
    lam = C.T @ Y
    full = np.zeros((n_mo, n_mo))
    full[:, :W] = lam
    G = 4.0 * (full - full.T)
    return lam, G


def lagrangian_direct(H, C, occ, b_half, b_mo, d, A, B):
    """The same lambda and G without the per-MO AO matrices.  Since b is
    symmetric, J^(r) c_q = sum_l d_lr b_half[q][l] and
    K^(r) c_q = sum_l b_mo[l][r][q] b_half[r][l], so

      Y[:, q] = n_q H c_q + sum_l a_lq b_half[q][l] + sum_{r,l} B_qr b_mo[l][r][q] b_half[r][l]
      with a_lq = sum_r A_qr d_lr,

    a contraction over (r, l) that never forms an n_bf x n_bf matrix per orbital.
    """
    W = occ.shape[0]
    n_mo = C.shape[1]
    a = d @ A.T                                              # a[l][q] = sum_r A_qr d_lr
    YJ = np.einsum("lq,qlm->mq", a, b_half)
    YK = np.einsum("qr,lrq,rlm->mq", B, b_mo, b_half)
    Y = occ[None, :] * (H @ C[:, :W]) + YJ + YK
    lam = C.T @ Y
    full = np.zeros((n_mo, n_mo))
    full[:, :W] = lam
    return lam, 4.0 * (full - full.T)


def build(b, C, H, occ, pair_of, n_pairs, functional="pnof7"):
    """All hot-path steps once: the unit of one build."""
    W = occ.shape[0]
    Co = np.ascontiguousarray(C[:, :W])
    bh = half_transform(b, Co)
    bmo = mo_transform(bh, Co)
    d = diag_of(bmo)
    J, K = jk_mo(bmo)
    Jn, Kn = jk_ao_per_mo(b, bh, d)
    Delta, Pi = delta_pi(occ, pair_of, n_pairs, functional)
    A, Bc = coefficients(occ, pair_of, n_pairs, functional)
    Hp = hpp(H, Co)
    E = energy(occ, Hp, J, K, Delta, Pi)
    lam, G = lagrangian(H, C, occ, Jn, Kn, A, Bc)
    return dict(b_half=bh, b_mo=bmo, d=d, J=J, K=K, Jn=Jn, Kn=Kn, A=A, B=Bc,
                Hpp=Hp, energy=E, lam=lam, grad=G)


def build_instance(inst, C=None, functional="pnof7"):
    return build(inst.b, inst.C if C is None else C, inst.H, inst.occ, inst.pair_of,
                 inst.n_pairs, functional)
