"""Pins of the ON optimiser and warm-start MLP oracles (CPU)."""
import numpy as np
import pytest

import synth
from oracle import mlp
from oracle import on_opt as on
from oracle import pnof7_ri as ri


def jk_instance(nb=14, na=40, npair=3, ncwo=2, seed=3):
    inst = synth.make_instance(nb, na, npair, ncwo, seed)
    o = ri.build_instance(inst)
    return inst, o["Hpp"], o["J"], o["K"]


@pytest.mark.parametrize("ncwo", [1, 2, 3])
def test_gamma_map(ncwo):
    npair = 3
    pm = synth.default_pair_map(npair, ncwo)
    rng = np.random.default_rng(ncwo)
    x = rng.uniform(0, np.pi / 2, npair * ncwo)
    n = on.gamma_to_n(x, pm, npair, ncwo)
    for g in range(npair):
        assert abs(n[pm == g].sum() - 1.0) < 1e-14
    assert np.all(n[:npair] >= 0.5) and np.all((n >= 0) & (n <= 1))
    assert np.allclose(on.gamma_to_n(on.n_to_gamma(n, pm, npair, ncwo), pm, npair, ncwo), n, atol=1e-13)
    n0 = on.gamma_to_n(on.cold_start(npair, ncwo), pm, npair, ncwo)
    assert np.allclose(n0[:npair], 0.98) and np.allclose(n0[npair:], 0.02 / ncwo)


@pytest.mark.parametrize("functional", ["pnof7", "pnof5"])
def test_grad_n_finite_difference(functional):
    inst, Hpp, J, K = jk_instance()
    rng = np.random.default_rng(1)
    n = rng.uniform(0.05, 0.95, inst.n_omega)
    g = on.grad_n(n, Hpp, J, K, inst.pair_of, inst.n_pairs, functional)
    h = 1e-6
    for p in range(inst.n_omega):
        e = np.zeros_like(n); e[p] = h
        fd = (on.energy_n(n + e, Hpp, J, K, inst.pair_of, inst.n_pairs, functional)
              - on.energy_n(n - e, Hpp, J, K, inst.pair_of, inst.n_pairs, functional)) / (2 * h)
        assert abs(fd - g[p]) < 1e-7 * max(1.0, abs(g[p])), p


@pytest.mark.parametrize("ncwo", [1, 2, 4])
def test_grad_gamma_finite_difference(ncwo):
    inst, Hpp, J, K = jk_instance(16, 45, 3, ncwo, 10 + ncwo)
    rng = np.random.default_rng(ncwo)
    x = rng.uniform(0.1, 1.4, inst.n_pairs * ncwo)
    g = on.grad_gamma(x, Hpp, J, K, inst.pair_of, inst.n_pairs, ncwo)
    h = 1e-6
    for i in range(len(x)):
        e = np.zeros_like(x); e[i] = h
        fd = (on.energy_gamma(x + e, Hpp, J, K, inst.pair_of, inst.n_pairs, ncwo)
              - on.energy_gamma(x - e, Hpp, J, K, inst.pair_of, inst.n_pairs, ncwo)) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(g[i])), i


@pytest.mark.parametrize("seed", [30, 31, 32])
def test_optimizer_two_electron_ci_limit(seed):
    """One pair, one weak orbital: the optimum is the lowest 2x2 CI eigenvalue
    (the strong orbital is chosen as the one the CI ground state occupies most,
    since the parametrisation keeps n_strong >= 1/2)."""
    inst = synth.make_instance(8, 20, 1, 1, seed)
    for _ in range(2):
        o = ri.build_instance(inst)
        Hpp, J, K = o["Hpp"], o["J"], o["K"]
        M = np.array([[2 * Hpp[0] + J[0, 0], K[0, 1]], [K[0, 1], 2 * Hpp[1] + J[1, 1]]])
        v = np.linalg.eigh(M)[1][:, 0]
        if v[0] ** 2 >= 0.5:
            break
        inst.C[:, [0, 1]] = inst.C[:, [1, 0]]
    x, E, nit, gmax = on.optimize(Hpp, J, K, inst.pair_of, 1, 1)
    assert gmax <= 1e-8
    assert abs(E - np.linalg.eigvalsh(M)[0]) < 1e-10


def test_optimizer_reaches_a_local_minimum():
    inst, Hpp, J, K = jk_instance(20, 60, 4, 3, 7)
    E0 = on.energy_gamma(on.cold_start(4, 3), Hpp, J, K, inst.pair_of, 4, 3)
    x, E, nit, gmax = on.optimize(Hpp, J, K, inst.pair_of, 4, 3)
    assert gmax <= 1e-8 and E < E0
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.standard_normal(len(x)) * 1e-3
        assert on.energy_gamma(x + d, Hpp, J, K, inst.pair_of, 4, 3) >= E - 1e-12


def test_mlp_backward_finite_difference():
    rng = np.random.default_rng(0)
    th = mlp.init_params(0) + 0.01 * rng.standard_normal(mlp.N_PARAMS)
    X = rng.standard_normal((5, mlp.N_IN))
    M = np.ones((5, mlp.N_OUT)); M[1, 4:] = 0; M[3, 2:] = 0
    T = rng.uniform(0, 1, (5, mlp.N_OUT)) * M
    p, cache = mlp.forward(th, X, M)
    assert np.allclose(p.sum(1), 1.0) and np.all(p[M == 0] == 0)
    g = mlp.backward(th, cache, T, M)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS); e[i] = h
        fd = (mlp.loss(mlp.forward(th + e, X, M)[0], T, M) - mlp.loss(mlp.forward(th - e, X, M)[0], T, M)) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 + 1e-5 * abs(g[i]), i


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-12)
    assert np.allclose(th[:3], -0.01 * np.sign(g[:3])) and th[3] == 0.0


def test_features_layout():
    inst, Hpp, J, K = jk_instance(20, 50, 3, 2, 4)
    X = mlp.features(Hpp, J, K, inst.pair_of, 3, 2)
    assert X.shape == (3, mlp.N_IN)
    assert np.all(X[:, 3 + 5 * 2: 3 + 5 * mlp.KMAX] == 0)              # empty slots
    assert np.all(X[:, 3 + 5 * mlp.KMAX:][:, :2] == 1) and np.all(X[:, 3 + 5 * mlp.KMAX + 2:] == 0)
    w0 = [p for p in range(3, inst.n_omega) if inst.pair_of[p] == 1][0]
    assert X[1, 5] == K[1, w0] and X[1, 0] == Hpp[1]
