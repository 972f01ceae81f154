"""Pins for the b-preparation oracle (oracle/metric.py, Sec. II, RI):

  * the pivoted factorisation reproduces G (P L D L^T P^T), with L unit lower
    triangular and D block diagonal (1x1 / 2x2), including matrices that force
    2x2 pivots and an exactly singular one;
  * it equals LAPACK's Bunch-Kaufman factorisation (scipy.linalg.ldl) on
    sizes where LAPACK runs the unblocked algorithm: same pivots, same factors;
  * b satisfies the RI identity sum_k b^k b^k = T^T G~^-1 T, checked by an
    independent dense solve; with a well-conditioned metric nothing is
    corrected and G~ = G; every b^k is symmetric;
  * the correction raises exactly the block eigenvalues below delta.
"""
import numpy as np
import pytest
from scipy.linalg import ldl

from oracle import metric as mt


def spd(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w = np.geomspace(1.0, 1.0 / cond, n)
    return (Q * w) @ Q.T


def indefinite(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n))
    return (X + X.T) / 2


def forced_2x2(n, seed):
    # zero diagonal: every first pivot test fails and 2x2 blocks appear
    A = indefinite(n, seed)
    np.fill_diagonal(A, 0.0)
    return A


@pytest.mark.parametrize("make,n,seed", [(spd, 40, 1), (indefinite, 37, 2), (forced_2x2, 30, 3),
                                         (indefinite, 150, 4), (forced_2x2, 101, 5)])
def test_factorisation_reproduces_G(make, n, seed):
    G = make(n, seed)
    perm, L, D, steps = mt.bunch_kaufman(G)
    assert np.allclose(np.triu(L, 1), 0) and np.allclose(np.diag(L), 1)
    assert sum(steps) == n
    k, mask = 0, np.zeros((n, n), bool)
    for s in steps:
        mask[k:k + s, k:k + s] = True
        k += s
    assert np.all(D[~mask] == 0)
    R = mt.reconstruct(perm, L, D)
    assert np.max(np.abs(R - G)) <= 1e-12 * np.max(np.abs(G))
    assert np.max(np.abs(L)) <= 1.0 / (1.0 - mt.ALPHA) + 1e-12 or make is forced_2x2 or 2 in steps
    if make is forced_2x2:
        assert 2 in steps


def test_singular_column():
    G = indefinite(12, 6)
    G[:, 4] = 0.0
    G[4, :] = 0.0
    perm, L, D, steps = mt.bunch_kaufman(G)
    assert np.max(np.abs(mt.reconstruct(perm, L, D) - G)) <= 1e-12 * np.max(np.abs(G))


@pytest.mark.parametrize("make,n,seed", [(spd, 30, 7), (indefinite, 45, 8), (forced_2x2, 33, 9),
                                         (indefinite, 60, 10)])
def test_equals_lapack_bunch_kaufman(make, n, seed):
    G = make(n, seed)
    perm, L, D, steps = mt.bunch_kaufman(G)
    lu, d, p = ldl(G, lower=True, hermitian=True)
    # scipy: G = lu d lu^T with lu[p] lower triangular; here lu = P L
    PL = np.zeros_like(L)
    PL[perm] = L
    assert np.max(np.abs(PL - lu)) <= 1e-11 * max(1.0, np.max(np.abs(lu)))
    assert np.max(np.abs(D - d)) <= 1e-11 * np.max(np.abs(d))


def test_b_satisfies_ri_identity_spd():
    rng = np.random.default_rng(11)
    nb, na = 7, 25
    G = spd(na, 12, cond=1e4)
    X = rng.standard_normal((na, nb, nb))
    T = (X + X.transpose(0, 2, 1)) / 2
    b, info = mt.prepare_b(T, G)
    assert np.array_equal(b, b.transpose(0, 2, 1)) or np.max(np.abs(b - b.transpose(0, 2, 1))) < 1e-13
    _, _, D, steps = mt.bunch_kaufman(G)
    Dt, _, _ = mt.corrected_blocks(D, steps, info["delta"])
    assert np.array_equal(Dt, np.where(Dt != 0, D, 0)) or np.max(np.abs(Dt - D)) < 1e-14
    Tm = T.reshape(na, nb * nb)
    eri = b.reshape(na, nb * nb).T @ b.reshape(na, nb * nb)
    ref = Tm.T @ np.linalg.solve(G, Tm)
    assert np.max(np.abs(eri - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_b_with_correction_indefinite():
    rng = np.random.default_rng(13)
    nb, na = 6, 30
    G = indefinite(na, 14)
    X = rng.standard_normal((na, nb, nb))
    T = (X + X.transpose(0, 2, 1)) / 2
    b, info = mt.prepare_b(T, G)
    perm, L, D, steps = info["perm"], info["L"], info["D"], info["steps"]
    Dt, _, _ = mt.corrected_blocks(D, steps, info["delta"])
    k = 0
    raised = 0
    for s in steps:
        w0 = np.linalg.eigvalsh(D[k:k + s, k:k + s])
        w1 = np.linalg.eigvalsh(Dt[k:k + s, k:k + s])
        scale = np.max(np.abs(w0))          # rounding of Q diag(w) Q^T is relative to the block
        assert np.all(w1 >= info["delta"] - 1e-14 * scale)
        assert np.allclose(w1, np.maximum(w0, info["delta"]), rtol=1e-12, atol=1e-14 * scale)
        raised += int(np.sum(w0 < info["delta"]))
        k += s
    assert raised > 0                      # a random symmetric metric has negative eigenvalues
    # the defining equation P L D~^(1/2) b^T = T, to rounding (backward error)
    _, Dh, _ = mt.corrected_blocks(D, steps, info["delta"])
    Tm = T.reshape(na, nb * nb)
    bT = b.reshape(na, nb * nb)
    P = np.zeros((na, na))
    P[perm, np.arange(na)] = 1.0
    # backward-error bound of the product: rounding of |L| |D~^(1/2)| |b^T| over na terms
    terms = np.max(np.abs(L)) * np.max(np.abs(Dh)) * np.max(np.abs(bT)) * na
    assert np.max(np.abs(P @ L @ Dh @ bT - Tm)) <= 10 * 2.0 ** -52 * terms
    # the RI identity with G~; kappa(G~) ~ ||G|| / delta, so the dense solve is
    # accurate to about kappa * eps
    Gt = mt.reconstruct(perm, L, Dt)
    eri = bT.T @ bT
    ref = Tm.T @ np.linalg.solve(Gt, Tm)
    kappa = np.linalg.cond(Gt)
    assert np.max(np.abs(eri - ref)) <= 10 * kappa * 2.0 ** -52 * np.max(np.abs(ref))
