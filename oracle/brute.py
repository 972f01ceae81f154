"""Independent brute-force routes that pin the RI oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Nothing here calls
into ``pnof7_ri``; these are the conventional, slower definitions the RI
algebra must reproduce exactly when the four-index integrals are built from
the same factors.

* ``eri4``:      (mu nu|sigma lambda) = sum_l b^l_{mu nu} b^l_{sigma lambda},
                 the fitted four-centre integral of Eq. (6) written with the
                 symmetric factor b of Eq. (9).
* ``table1``:    the conventional algorithm of Table 1 (Eqs. (3)-(5)).
* ``rhf``:       closed-shell Fock matrix and energy from a density matrix
                 (textbook Hartree-Fock, used for the occupation 0/1 limit).
* ``apsg_expectation``: <Psi|H|Psi> for an antisymmetrised product of
                 strongly orthogonal singlet geminals written in natural
                 orbitals, evaluated by applying second-quantised operators
                 to determinants.  PNOF5 (the functional the paper notes is
                 strictly pure N-representable) equals this expectation value.
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = ["eri4", "table1", "mo_eri", "rhf", "apsg_expectation"]


def eri4(b: np.ndarray) -> np.ndarray:
    A, B, _ = b.shape
    X = b.reshape(A, B * B)
    return (X.T @ X).reshape(B, B, B, B)


def table1(eri: np.ndarray, C_omega: np.ndarray):
    """Table 1, steps 1-3.  Returns J, K (MO) and Jq, Kq (per-MO AO)."""
    W = C_omega.shape[1]
    B = C_omega.shape[0]
    Jq = np.empty((W, B, B))
    Kq = np.empty((W, B, B))
    for q in range(W):
        Pq = np.outer(C_omega[:, q], C_omega[:, q])             # Eq. (4)
        Jq[q] = np.einsum("mnsl,sl->mn", eri, Pq)               # step 2, J branch
        Kq[q] = np.einsum("mnsl,nl->ms", eri, Pq)               # step 2, K branch
    J = np.empty((W, W))
    K = np.empty((W, W))
    for p in range(W):
        Pp = np.outer(C_omega[:, p], C_omega[:, p])
        for q in range(W):
            J[p, q] = np.sum(Pp * Jq[q])                       # Eq. (3)
            K[p, q] = np.sum(Pp * Kq[q])                       # Eq. (5)
    return J, K, Jq, Kq


def mo_eri(eri: np.ndarray, Cm: np.ndarray) -> np.ndarray:
    """(pq|rs) = sum C_mu p C_nu q C_sigma r C_lambda s (mu nu|sigma lambda)."""
    t = np.einsum("mnsl,mp->pnsl", eri, Cm)
    t = np.einsum("pnsl,nq->pqsl", t, Cm)
    t = np.einsum("pqsl,sr->pqrl", t, Cm)
    return np.einsum("pqrl,ls->pqrs", t, Cm)


def rhf(eri: np.ndarray, H: np.ndarray, C_occ: np.ndarray):
    """Closed-shell HF: D = C_occ C_occ^T, F = H + 2 J[D] - K[D], E = tr D (H + F)."""
    D = C_occ @ C_occ.T
    Jd = np.einsum("mnsl,sl->mn", eri, D)
    Kd = np.einsum("mnsl,nl->ms", eri, D)
    F = H + 2.0 * Jd - Kd
    return float(np.sum(D * (H + F))), F


# ---- second quantisation on bit-string determinants -------------------------
# spin orbital 2p is p-alpha, 2p+1 is p-beta.

def _apply_create(det: int, i: int):
    if det >> i & 1:
        return None, 0
    sign = -1 if bin(det & ((1 << i) - 1)).count("1") & 1 else 1
    return det | (1 << i), sign


def _apply_annihilate(det: int, i: int):
    if not det >> i & 1:
        return None, 0
    sign = -1 if bin(det & ((1 << i) - 1)).count("1") & 1 else 1
    return det & ~(1 << i), sign


def _apply_string(ops, det):
    """Apply operators right-to-left; ops is a list of (kind, index), leftmost first."""
    sign = 1
    for kind, i in reversed(ops):
        det, s = (_apply_create if kind == "c" else _apply_annihilate)(det, i)
        if det is None:
            return None, 0
        sign *= s
    return det, sign


def apsg_state(groups, coef):
    """Psi = prod_g (sum_{p in group g} coef[p] a+_{p alpha} a+_{p beta}) |vac>."""
    state = {0: 1.0}
    for grp in groups:
        new = {}
        for det, c in state.items():
            for p in grp:
                d2, s = _apply_string([("c", 2 * p), ("c", 2 * p + 1)], det)
                if d2 is None:
                    continue
                new[d2] = new.get(d2, 0.0) + s * c * coef[p]
        state = new
    return state


def apply_hamiltonian(h: np.ndarray, g: np.ndarray, state: dict) -> dict:
    """H = sum h_pq a+_{p s} a_{q s} + 1/2 sum (pq|rs) a+_{p s} a+_{r t} a_{s t} a_{q s}."""
    n = h.shape[0]
    out = {}
    for det, c in state.items():
        for p, q in itertools.product(range(n), repeat=2):
            if h[p, q] == 0.0:
                continue
            for s in (0, 1):
                d2, sg = _apply_string([("c", 2 * p + s), ("a", 2 * q + s)], det)
                if d2 is not None:
                    out[d2] = out.get(d2, 0.0) + sg * c * h[p, q]
        for p, q, r, s_ in itertools.product(range(n), repeat=4):
            v = g[p, q, r, s_]
            if v == 0.0:
                continue
            for s, t in itertools.product((0, 1), repeat=2):
                d2, sg = _apply_string([("c", 2 * p + s), ("c", 2 * r + t),
                                        ("a", 2 * s_ + t), ("a", 2 * q + s)], det)
                if d2 is not None:
                    out[d2] = out.get(d2, 0.0) + 0.5 * sg * c * v
    return out


def apsg_expectation(h_mo: np.ndarray, g_mo: np.ndarray, occ: np.ndarray,
                     pair_of: np.ndarray, n_pairs: int) -> float:
    """<Psi|H|Psi>/<Psi|Psi> for the geminal product whose natural orbitals are
    the orbitals of Omega with occupations occ: the strong orbital g of pair g
    carries +sqrt(n_g), each weak orbital -sqrt(n_p)."""
    W = occ.shape[0]
    coef = np.where(np.arange(W) < n_pairs, np.sqrt(occ), -np.sqrt(occ))
    groups = [[p for p in range(W) if pair_of[p] == g] for g in range(n_pairs)]
    psi = apsg_state(groups, coef)
    hpsi = apply_hamiltonian(h_mo, g_mo, psi)
    num = sum(c * hpsi.get(d, 0.0) for d, c in psi.items())
    den = sum(c * c for c in psi.values())
    return num / den
