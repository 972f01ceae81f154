"""Pins for the orbital-optimisation oracle (iterative diagonalisation of
F^lambda, Sec. II) and the outer/inner loop of Fig. 1, against facts that do
not come from the oracle itself:

  * first-order descent: with a steep ascending diagonal, one step changes the
    energy by -4 sum_{q<p} (lambda_qp - lambda_pq)^2 / (eps_p - eps_q)
    (perturbation theory of the eigenvectors); a sign or transpose error in
    F^lambda flips or scrambles this;
  * without two-electron terms the energy is 2 sum_p n_p c_p^T H c_p, whose
    minimum over orthonormal orbitals is 2 sum_p n_p eps_p with the ONs
    descending and the eigenvalues of H ascending (rearrangement / von
    Neumann trace bound);
  * a converged point is stationary with non-negative curvature;
  * two electrons in one pair that spans every orbital: PNOF7 is then the
    energy of a normalised two-electron singlet, so it never goes below full
    CI, and at the FCI natural orbitals and ONs it equals full CI (when the
    FCI natural-orbital coefficients have one sign for the strong orbital and
    the other for all weak ones), with a zero orbital gradient; from those
    orbitals with other ONs the loop's ON step returns to full CI.  Full CI here
    is brute-force diagonalisation in the space of symmetric two-electron
    spatial functions.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import orbital as orb
from oracle import pnof7_ri as ri


@pytest.fixture(scope="module")
def small():
    inst = synth.make_instance(12, 36, 3, 1, 7)
    occ = np.array([0.99, 0.97, 0.95, 0.05, 0.03, 0.01])   # descending along Omega
    return inst, occ


def test_fock_lambda_shape(small):
    inst, occ = small
    r = ri.build(inst.b, inst.C, inst.H, occ, inst.pair_of, inst.n_pairs)
    F = orb.fock_lambda(r["lam"], inst.n_mo)
    assert np.array_equal(F, F.T)
    L = orb.lambda_full(r["lam"], inst.n_mo)
    off = F - np.diag(np.diag(F))
    # |F_pq| = |G_pq| / 4 off the diagonal, and F's diagonal is lambda_pp
    assert np.allclose(np.abs(off), np.abs(r["grad"]) / 4, rtol=0, atol=1e-14)
    assert np.array_equal(np.diag(F), np.diag(L))
    # lambda symmetric on Omega and zero for rows outside it -> F is diagonal
    X = np.random.default_rng(3).standard_normal((occ.size, occ.size))
    lam = np.zeros((inst.n_mo, occ.size))
    lam[:occ.size] = X + X.T
    Fs = orb.fock_lambda(lam, inst.n_mo)
    assert np.array_equal(Fs, np.diag(np.diag(Fs)))


def test_descent_matches_first_order(small):
    inst, occ = small
    n = inst.n_mo
    r = ri.build(inst.b, inst.C, inst.H, occ, inst.pair_of, inst.n_pairs)
    L = orb.lambda_full(r["lam"], n)
    for scale, rel in ((1e3, 2e-3), (1e4, 2e-4)):
        eps = scale * np.arange(n)
        C1, w = orb.orbital_step(inst.C, r["lam"], eps)
        dE = ri.build(inst.b, C1, inst.H, occ, inst.pair_of, inst.n_pairs)["energy"] - r["energy"]
        pred = -4 * sum((L[q, p] - L[p, q]) ** 2 / (eps[p] - eps[q])
                        for q in range(n) for p in range(q + 1, n))
        assert pred < 0 and dE < 0
        assert abs(dE - pred) <= rel * abs(pred), (scale, dE, pred)
        assert np.allclose(C1.T @ C1, np.eye(n), atol=1e-13)


def test_no_two_electron_terms_reach_trace_minimum(small):
    inst, occ = small
    b0 = np.zeros_like(inst.b)
    res = orb.inner_loop(b0, inst.C, inst.H, occ, inst.pair_of, inst.n_pairs, 3000, 1e-10)
    eh = np.linalg.eigvalsh(inst.H)
    e_min = 2 * np.sum(np.sort(occ)[::-1] * eh[:occ.size])
    assert abs(res["energies"][-1] - e_min) <= 1e-9 * abs(e_min)
    assert min(res["energies"]) >= e_min - 1e-9 * abs(e_min)
    assert np.allclose(res["C"].T @ res["C"], np.eye(inst.n_mo), atol=1e-12)


def test_converged_point_is_a_local_minimum(small):
    inst, occ = small
    res = orb.inner_loop(inst.b, inst.C, inst.H, occ, inst.pair_of, inst.n_pairs, 5000, 1e-9)
    assert res["converged"] and res["grads"][-1] <= 1e-9
    assert res["energies"][-1] < res["energies"][0]
    C, E = res["C"], res["energies"][-1]
    rng = np.random.default_rng(1)
    for _ in range(10):
        X = rng.standard_normal((inst.n_mo, inst.n_mo))
        k = (X - X.T) / 2
        Es = ri.build(inst.b, C @ expm(1e-2 * k), inst.H, occ, inst.pair_of, inst.n_pairs)["energy"]
        assert Es >= E - 1e-12


def fci_two_electrons(h, eri):
    """Lowest singlet of two electrons: Psi(1,2) = sum_pq X_pq phi_p(1) phi_q(2),
    X symmetric, <Psi|h1 + h2 + 1/r12|Psi> with (pr|qs) = eri[p,r,q,s]."""
    n = h.shape[0]
    I = np.eye(n)
    M = (np.einsum("pr,qs->pqrs", h, I) + np.einsum("pr,qs->pqrs", I, h)
         + np.einsum("prqs->pqrs", eri)).reshape(n * n, n * n)
    basis = []
    for p in range(n):
        for q in range(p, n):
            v = np.zeros((n, n))
            v[p, q] = v[q, p] = 1.0
            basis.append(v.ravel() / np.linalg.norm(v))
    S = np.array(basis).T
    w, U = np.linalg.eigh(S.T @ M @ S)
    return w[0], (S @ U[:, 0]).reshape(n, n)


@pytest.mark.parametrize("seed", [103, 104, 105, 106, 107])
def test_two_electron_full_ci(seed):
    nb = 5
    inst = synth.make_instance(nb, 3 * nb, 1, nb - 1, seed)
    h = inst.C.T @ inst.H @ inst.C
    bm = np.einsum("mp,lmn,nq->lpq", inst.C, inst.b, inst.C)
    e_fci, X = fci_two_electrons(h, np.einsum("lpq,lrs->pqrs", bm, bm))
    c, U = np.linalg.eigh(X)
    order = np.argsort(-np.abs(c))
    c, U = c[order], U[:, order]
    c = c if c[0] > 0 else -c
    C0, occ = inst.C @ U, c ** 2
    r = ri.build(inst.b, C0, inst.H, occ, inst.pair_of, 1)
    loop = orb.outer_loop(inst.b, C0, inst.H, occ, inst.pair_of, 1, nb - 1, 5, 50, 1e-8, 1e-11)
    if np.all(c[1:] < 0):
        assert abs(r["energy"] - e_fci) <= 1e-12 * abs(e_fci)
        assert np.max(np.abs(r["grad"])) <= 1e-12
        assert loop["converged"] and abs(loop["energies"][-1] - e_fci) <= 1e-12 * abs(e_fci)
        # same orbitals, wrong ONs: the ON step of the first outer iteration
        # must bring the energy back to full CI
        bad = np.full(nb, 0.1 / (nb - 1))
        bad[0] = 0.9
        loop2 = orb.outer_loop(inst.b, C0, inst.H, bad, inst.pair_of, 1, nb - 1, 5, 50, 1e-8, 1e-11)
        assert abs(loop2["energies"][-1] - e_fci) <= 1e-10 * abs(e_fci)
    else:
        assert r["energy"] > e_fci + 1e-6
    assert min(loop["energies"]) >= e_fci - 1e-12 * abs(e_fci)
