"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself:
  * brute force over the explicit four-index integrals with the conventional
    algorithm of Table 1 (the RI path must reproduce it exactly, since the
    four-index tensor is built from the same factors);
  * the closed-shell Hartree-Fock limit (occupations 0/1), built by an
    independent density-matrix route;
  * the expectation value of an antisymmetrised geminal product, which PNOF5
    (PNOF7 without its inter-pair Phi term) reproduces exactly;
  * finite differences of the energy along orbital rotations;
  * invariances and the identities listed with each test.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import brute, pnof7_ri as ri


def small(n_bf=14, n_aux=40, n_pairs=2, n_cwo=2, seed=5, n_mo=None):
    return synth.make_instance(n_bf, n_aux, n_pairs, n_cwo, seed, n_mo=n_mo)


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("shape", [(12, 30, 2, 1, 0), (17, 23, 2, 2, 1), (20, 61, 3, 2, 2),
                                   (9, 5, 1, 3, 3)])
def test_ri_equals_table1_bruteforce(shape):
    nb, na, npair, ncwo, seed = shape
    inst = small(nb, na, npair, ncwo, seed)
    W = inst.n_omega
    Co = inst.C[:, :W]
    out = ri.build_instance(inst)
    J4, K4, Jq4, Kq4 = brute.table1(brute.eri4(inst.b), Co)
    assert rel(out["J"], J4) < 1e-12
    assert rel(out["K"], K4) < 1e-12
    assert rel(out["Jn"], Jq4) < 1e-12
    assert rel(out["Kn"], Kq4) < 1e-12


def test_transform_definitions_against_loops():
    inst = small(7, 9, 1, 2, 11)
    W = inst.n_omega
    Co = inst.C[:, :W]
    bh = ri.half_transform(inst.b, Co)
    bmo = ri.mo_transform(bh, Co)
    for q in range(W):
        for l in range(inst.n_aux):
            for nu in range(inst.n_bf):
                s = sum(Co[mu, q] * inst.b[l, mu, nu] for mu in range(inst.n_bf))
                assert abs(s - bh[q, l, nu]) < 1e-13
    for l in range(inst.n_aux):
        for p in range(W):
            for q in range(W):
                s = sum(Co[nu, q] * bh[p, l, nu] for nu in range(inst.n_bf))
                assert abs(s - bmo[l, p, q]) < 1e-13


def test_invariants():
    inst = small(22, 50, 3, 2, 7)
    W = inst.n_omega
    Co = inst.C[:, :W]
    o = ri.build_instance(inst)
    J, K, Jn, Kn = o["J"], o["K"], o["Jn"], o["Kn"]
    assert np.allclose(J, J.T, atol=1e-14, rtol=0)
    assert np.allclose(K, K.T, atol=1e-14, rtol=0)
    assert np.allclose(np.diag(J), np.diag(K), rtol=1e-13, atol=0)
    assert np.all(K >= 0)
    assert np.all(np.abs(J) <= np.sqrt(np.outer(np.diag(J), np.diag(J))) * (1 + 1e-13))
    for n in range(W):
        assert np.allclose(Jn[n], Jn[n].T, atol=1e-14)
        assert np.allclose(Kn[n], Kn[n].T, atol=1e-14)
        # c_m^T J^(n) c_m = J_mn, c_m^T K^(n) c_m = K_mn
        assert np.allclose(np.einsum("mi,mn,ni->i", Co, Jn[n], Co), J[:, n], rtol=1e-12, atol=1e-14)
        assert np.allclose(np.einsum("mi,mn,ni->i", Co, Kn[n], Co), K[:, n], rtol=1e-12, atol=1e-14)
        # J^(n) c_n = K^(n) c_n
        assert np.allclose(Jn[n] @ Co[:, n], Kn[n] @ Co[:, n], rtol=1e-12, atol=1e-14)
        assert np.linalg.eigvalsh(Kn[n]).min() > -1e-13
    # per-pair ON sums are 1, every ON in [0, 1]
    for g in range(inst.n_pairs):
        assert abs(inst.occ[inst.pair_of == g].sum() - 1.0) < 1e-15
    assert np.all((inst.occ >= 0) & (inst.occ <= 1))


def test_energy_lambda_identity_and_zero_columns():
    inst = small(16, 35, 2, 3, 9)
    o = ri.build_instance(inst)
    W = inst.n_omega
    E2 = np.sum(inst.occ * o["Hpp"]) + np.trace(o["lam"][:W, :W])
    assert abs(E2 - o["energy"]) < 1e-12 * abs(o["energy"])
    assert np.allclose(o["grad"], -o["grad"].T, atol=0)
    # regrouped coefficients reproduce Eq. (2) term by term
    Delta, Pi = ri.delta_pi(inst.occ, inst.pair_of, inst.n_pairs)
    A, B = ri.coefficients(inst.occ, inst.pair_of, inst.n_pairs)
    Ea = ri.energy_from_coefficients(inst.occ, o["Hpp"], o["J"], o["K"], A, B)
    assert abs(Ea - o["energy"]) < 1e-12 * abs(Ea)


def test_aux_rotation_invariance():
    inst = small(13, 29, 2, 1, 3)
    O, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((inst.n_aux, inst.n_aux)))
    b2 = np.einsum("kl,lmn->kmn", O, inst.b)
    o1 = ri.build_instance(inst)
    o2 = ri.build(b2, inst.C, inst.H, inst.occ, inst.pair_of, inst.n_pairs)
    for key in ("J", "K", "Jn", "Kn", "grad", "lam"):
        assert rel(o2[key], o1[key]) < 1e-12, key
    assert abs(o2["energy"] - o1["energy"]) < 1e-12 * abs(o1["energy"])


def test_ao_rotation_invariance():
    inst = small(15, 33, 2, 2, 4)
    R, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((inst.n_bf, inst.n_bf)))
    b2 = np.einsum("mi,lmn,nj->lij", R, inst.b, R)
    C2 = R.T @ inst.C
    H2 = R.T @ inst.H @ R
    o1 = ri.build_instance(inst)
    o2 = ri.build(b2, C2, H2, inst.occ, inst.pair_of, inst.n_pairs)
    for key in ("J", "K", "grad", "lam"):
        assert rel(o2[key], o1[key]) < 1e-12, key
    assert rel(o2["Jn"], np.einsum("mi,qmn,nj->qij", R, o1["Jn"], R)) < 1e-12
    assert rel(o2["Kn"], np.einsum("mi,qmn,nj->qij", R, o1["Kn"], R)) < 1e-12
    assert abs(o2["energy"] - o1["energy"]) < 1e-12 * abs(o1["energy"])


def test_column_sign_flip():
    inst = small(14, 31, 2, 2, 6)
    s = np.where(np.random.default_rng(2).random(inst.n_mo) < 0.5, -1.0, 1.0)
    o1 = ri.build_instance(inst)
    o2 = ri.build_instance(inst, C=inst.C * s[None, :])
    assert rel(o2["J"], o1["J"]) < 1e-13 and rel(o2["K"], o1["K"]) < 1e-13
    assert abs(o2["energy"] - o1["energy"]) < 1e-13 * abs(o1["energy"])
    assert rel(o2["grad"], o1["grad"] * np.outer(s, s)) < 1e-12


def test_hartree_fock_limit():
    """occ in {0, 1}: the energy is the closed-shell HF energy tr D(H+F) and
    the occupied-virtual gradient block is 4 F_ai."""
    inst = small(18, 45, 3, 2, 8)
    occ = np.where(np.arange(inst.n_omega) < inst.n_pairs, 1.0, 0.0)
    o = ri.build(inst.b, inst.C, inst.H, occ, inst.pair_of, inst.n_pairs)
    Cocc = inst.C[:, :inst.n_pairs]
    E_hf, F = brute.rhf(brute.eri4(inst.b), inst.H, Cocc)
    assert abs(o["energy"] - E_hf) < 1e-12 * abs(E_hf)
    Fmo = inst.C.T @ F @ inst.C
    P = inst.n_pairs
    G = o["grad"]
    assert rel(G[P:, :P], 4.0 * Fmo[P:, :P]) < 1e-12
    assert np.max(np.abs(G[:P, :P])) < 1e-12 * np.max(np.abs(G))


@pytest.mark.parametrize("shape", [(2, 1, 0), (2, 2, 1), (3, 1, 2), (1, 3, 3)])
def test_pnof5_equals_geminal_product_expectation(shape):
    """PNOF5 is the energy of an antisymmetrised product of strongly orthogonal
    geminals; evaluate <Psi|H|Psi> by second quantisation and compare."""
    npair, ncwo, seed = shape
    inst = small(10, 25, npair, ncwo, 20 + seed)
    W = inst.n_omega
    Co = inst.C[:, :W]
    rng = np.random.default_rng(seed)
    occ = inst.occ.copy()
    for g in range(npair):   # non-uniform weak ONs, still summing to 1 per pair
        idx = np.where(inst.pair_of == g)[0]
        w = rng.uniform(0.1, 1.0, len(idx)); w[0] = 3.0 * len(idx)
        occ[idx] = w / w.sum()
    o = ri.build(inst.b, inst.C, inst.H, occ, inst.pair_of, npair, functional="pnof5")
    h_mo = Co.T @ inst.H @ Co
    g_mo = brute.mo_eri(brute.eri4(inst.b), Co)
    E_ref = brute.apsg_expectation(h_mo, g_mo, occ, inst.pair_of, npair)
    assert abs(o["energy"] - E_ref) < 1e-12 * max(1.0, abs(E_ref))


def test_two_electron_minimum_is_ci_eigenvalue():
    """One pair, one weak orbital: minimising over the ON gives the lowest
    eigenvalue of the 2x2 CI matrix over the two closed-shell configurations."""
    from scipy.optimize import minimize_scalar
    inst = small(8, 20, 1, 1, 30)
    o = ri.build_instance(inst)
    Hpp, J, K = o["Hpp"], o["J"], o["K"]
    M = np.array([[2 * Hpp[0] + J[0, 0], K[0, 1]], [K[0, 1], 2 * Hpp[1] + J[1, 1]]])
    e0 = np.linalg.eigvalsh(M)[0]

    def E(x):
        n = np.array([x, 1.0 - x])
        return ri.energy(n, Hpp, J, K, *ri.delta_pi(n, inst.pair_of, 1))

    grid = np.linspace(0.0, 1.0, 2001)
    vals = np.array([E(x) for x in grid])
    i = int(np.argmin(vals))
    res = minimize_scalar(E, bounds=(grid[max(i - 1, 0)], grid[min(i + 1, 2000)]),
                          method="bounded", options={"xatol": 1e-13})
    assert vals.min() >= e0 - 1e-12
    assert abs(res.fun - e0) < 1e-10


@pytest.mark.parametrize("ab", [(0, 3), (1, 5), (2, 9), (4, 11), (6, 13), (12, 3)])
def test_gradient_finite_difference(ab):
    inst = small(15, 34, 2, 2, 12)
    o = ri.build_instance(inst)
    a, b_ = ab
    def E(theta):
        X = np.zeros((inst.n_mo, inst.n_mo)); X[a, b_] = theta; X[b_, a] = -theta
        return ri.build_instance(inst, C=inst.C @ expm(X))["energy"]
    h = 1e-4
    fd = (8 * (E(h) - E(-h)) - (E(2 * h) - E(-2 * h))) / (12 * h)
    assert abs(fd - o["grad"][a, b_]) < 1e-8 * max(1.0, np.max(np.abs(o["grad"])))


def test_pnof7_phi_term_vanishes_at_integer_occupations():
    inst = small(12, 30, 3, 1, 40)
    occ = np.where(np.arange(inst.n_omega) < inst.n_pairs, 1.0, 0.0)
    o7 = ri.build(inst.b, inst.C, inst.H, occ, inst.pair_of, inst.n_pairs, "pnof7")
    o5 = ri.build(inst.b, inst.C, inst.H, occ, inst.pair_of, inst.n_pairs, "pnof5")
    assert o7["energy"] == pytest.approx(o5["energy"], rel=1e-15)


@pytest.mark.parametrize("shape", [(15, 34, 2, 2, 12), (20, 17, 3, 1, 41), (9, 40, 1, 3, 42)])
def test_direct_lagrangian_equals_per_mo_route_and_finite_differences(shape):
    """The gradient path without per-MO AO matrices gives the lambda and G of
    the J^(n)/K^(n) route, and its G matches finite differences of the energy
    along orbital rotations (n_mo > n_omega rows included)."""
    inst = small(*shape)
    o = ri.build_instance(inst)
    lam, G = ri.lagrangian_direct(inst.H, inst.C, inst.occ, o["b_half"], o["b_mo"], o["d"], o["A"], o["B"])
    assert np.max(np.abs(lam - o["lam"])) <= 1e-12 * np.max(np.abs(o["lam"]))
    assert np.max(np.abs(G - o["grad"])) <= 1e-12 * np.max(np.abs(o["grad"]))
    n = inst.n_mo
    rng = np.random.default_rng(shape[-1])
    for _ in range(3):
        a, b_ = sorted(rng.choice(n, 2, replace=False))
        def E(theta):
            X = np.zeros((n, n)); X[a, b_] = theta; X[b_, a] = -theta
            return ri.build_instance(inst, C=inst.C @ expm(X))["energy"]
        h = 1e-4
        fd = (8 * (E(h) - E(-h)) - (E(2 * h) - E(-2 * h))) / (12 * h)
        assert abs(fd - G[a, b_]) < 1e-8 * max(1.0, np.max(np.abs(G)))
