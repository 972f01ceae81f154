"""ON optimiser, features, MLP and Adam kernels vs the FP64 oracle, and the
gain of the trained warm start over the cold start."""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle import on_opt as oon
from oracle import pnof7_ri as ri
from tests.gpu_util import host, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    c = rif.Context()
    yield c
    c.close()


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).cuda()


def problem(inst):
    """Oracle J, K, H_pp of an instance, uploaded (the optimiser's inputs)."""
    import torch
    o = ri.build_instance(inst)
    return o, (dev(o["Hpp"]), dev(o["J"]), dev(o["K"]), dev(inst.pair_of.astype(np.int32)),
               inst.n_pairs, inst.n_cwo)


def cold(ctx, onset):
    from paper_2012_15662_amd import warmstart as ws
    return ws.solve(ctx, onset, ws.prior_rows(onset))


SHAPES = [(20, 60, 2, 1, 1), (24, 72, 2, 2, 2), (30, 90, 3, 3, 3), (36, 100, 3, 2, 4), (40, 120, 3, 4, 5)]


def test_on_optimize_matches_oracle(ctx):
    import paper_2012_15662_amd as rif
    insts = [synth.make_instance(*s) for s in SHAPES]
    probs = [problem(i) for i in insts]
    onset = rif.OnSet(ctx, [p[1] for p in probs], tol=1e-8)
    it, st, _ = cold(ctx, onset)
    assert np.all(st == 0), st
    E = host(onset.energy)
    gam = host(onset.gamma)
    occ = host(onset.occ)
    for k, (inst, (o, _)) in enumerate(zip(insts, probs)):
        print(f"case n_bf={inst.n_bf} pairs={inst.n_pairs} ncwo={inst.n_cwo} gpu_iters={it[k]}", flush=True)
        x_ref, E_ref, nit, gmax = oon.optimize(o["Hpp"], o["J"], o["K"], inst.pair_of, inst.n_pairs, inst.n_cwo)
        xg = gam[onset.gslices[k]]
        # the GPU optimum is a stationary point by the oracle's own gradient ...
        g = oon.grad_gamma(xg, o["Hpp"], o["J"], o["K"], inst.pair_of, inst.n_pairs, inst.n_cwo)
        assert np.max(np.abs(g)) < 1e-7
        # ... with the oracle energy at those variables, and the same minimum
        Eg = oon.energy_gamma(xg, o["Hpp"], o["J"], o["K"], inst.pair_of, inst.n_pairs, inst.n_cwo)
        assert abs(E[k] - Eg) < 1e-12 * abs(Eg)
        assert abs(E[k] - E_ref) < 1e-10 * abs(E_ref)
        n_ref = oon.gamma_to_n(x_ref, inst.pair_of, inst.n_pairs, inst.n_cwo)
        assert np.max(np.abs(occ[onset.oslices[k]] - n_ref)) < 1e-5


def test_on_optimize_two_electron_ci(ctx):
    import paper_2012_15662_amd as rif
    inst = synth.make_instance(8, 20, 1, 1, 31)
    o = ri.build_instance(inst)
    M = np.array([[2 * o["Hpp"][0] + o["J"][0, 0], o["K"][0, 1]], [o["K"][0, 1], 2 * o["Hpp"][1] + o["J"][1, 1]]])
    if np.linalg.eigh(M)[1][0, 0] ** 2 < 0.5:
        inst.C[:, [0, 1]] = inst.C[:, [1, 0]]
        o = ri.build_instance(inst)
        M = M[::-1, ::-1]
    _, p = problem(inst)
    onset = rif.OnSet(ctx, [p])
    it, st, _ = cold(ctx, onset)
    assert st[0] == 0
    assert abs(host(onset.energy)[0] - np.linalg.eigvalsh(M)[0]) < 1e-10


def test_features_match_oracle(ctx):
    import paper_2012_15662_amd as rif
    from paper_2012_15662_amd import warmstart as ws
    insts = [synth.make_instance(*s) for s in SHAPES]
    probs = [problem(i) for i in insts]
    onset = rif.OnSet(ctx, [p[1] for p in probs])
    cold(ctx, onset)
    X, T, M = ws.features(ctx, onset, with_targets=True)
    X, T, M = host(X), host(T), host(M)
    occ = host(onset.occ)
    r = 0
    for k, (inst, (o, _)) in enumerate(zip(insts, probs)):
        Xr = omlp.features(o["Hpp"], o["J"], o["K"], inst.pair_of, inst.n_pairs, inst.n_cwo)
        Tr, Mr = omlp.targets(occ[onset.oslices[k]], inst.pair_of, inst.n_pairs)
        n = inst.n_pairs
        assert np.allclose(X[r:r + n], Xr, rtol=1e-6, atol=1e-6)
        assert np.allclose(T[r:r + n], Tr, rtol=1e-6, atol=1e-7) and np.array_equal(M[r:r + n], Mr)
        r += n


def test_mlp_forward_backward_adam_vs_oracle(ctx):
    import torch
    rng = np.random.default_rng(0)
    n = 300
    th = (omlp.init_params(1) + 0.05 * rng.standard_normal(omlp.N_PARAMS)).astype(np.float32)
    X = rng.standard_normal((n, omlp.N_IN)).astype(np.float32)
    M = np.ones((n, omlp.N_OUT), np.float32)
    M[rng.random((n, omlp.N_OUT)) < 0.3] = 0
    M[:, 0] = 1
    T = (rng.random((n, omlp.N_OUT)) * M).astype(np.float32)
    assert ctx.mlp_n_params() == omlp.N_PARAMS
    f = torch.float32
    tX, tM, tT, tth = dev(X), dev(M), dev(T), dev(th)
    H = torch.empty((3, n, 128), dtype=f, device="cuda")
    Z = torch.empty((n, 7), dtype=f, device="cuda")
    P = torch.empty((n, 7), dtype=f, device="cuda")
    dA = torch.empty((2, n, 128), dtype=f, device="cuda")
    g = torch.empty_like(tth)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.mlp_forward(tX, tM, tth, H, Z, P)
    ctx.mlp_backward(tX, tM, tT, tth, H, Z, dA, g, loss)
    ctx.sync()
    p_ref, cache = omlp.forward(th.astype(np.float64), X.astype(np.float64), M.astype(np.float64))
    g_ref = omlp.backward(th.astype(np.float64), cache, T.astype(np.float64), M.astype(np.float64))
    print("P", relerr(host(P), p_ref), "grad", relerr(host(g), g_ref), flush=True)
    assert relerr(host(P), p_ref) < 1e-5
    assert relerr(host(g), g_ref) < 1e-4
    assert abs(host(loss)[0] - omlp.loss(p_ref, T, M)) < 1e-5 * omlp.loss(p_ref, T, M)
    m = torch.zeros_like(tth)
    v = torch.zeros_like(tth)
    gr = host(g).astype(np.float64)
    th_ref, m_ref, v_ref = th.astype(np.float64), np.zeros(omlp.N_PARAMS), np.zeros(omlp.N_PARAMS)
    for step in (1, 2, 3):
        ctx.adam(tth, g, m, v, step, 1e-3)
        th_ref, m_ref, v_ref = omlp.adam_step(th_ref, gr, m_ref, v_ref, step, 1e-3)
    ctx.sync()
    assert relerr(host(tth), th_ref) < 1e-6


def test_trained_warm_start_cuts_iterations(ctx):
    """Train on molecules the method itself solves, then start held-out
    molecules from the network's ONs: fewer ON iterations, same minima."""
    import paper_2012_15662_amd as rif
    from paper_2012_15662_amd import warmstart as ws
    rng = np.random.default_rng(7)
    def batch(n, seed0):
        out = []
        for i in range(n):
            nb = int(rng.integers(24, 61))
            ncwo = int(rng.integers(1, 4))
            inp, npair, nc = synth.make_instance_device(nb, 3 * nb, max(1, nb // 12), ncwo, seed0 + i)
            out.append(ws.jk_problem(ctx, inp, npair, nc))
        return out
    train, test = batch(120, 100), batch(30, 900)
    tr = rif.OnSet(ctx, train)
    it_tr, st_tr, _ = cold(ctx, tr)
    X, T, M = ws.features(ctx, tr, with_targets=True)
    mu, sd = ws.standardisation(X)
    X, T, M = ws.features(ctx, tr, with_targets=True, mu=mu, sigma=sd)
    net = ws.WarmStartMLP(ctx, seed=0)
    losses = net.fit(X, T, M, epochs=600, lr=3e-3)
    print("loss", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.2 * losses[0]
    te_cold = rif.OnSet(ctx, test)
    it_c, st_c, _ = cold(ctx, te_cold)
    te_warm = rif.OnSet(ctx, test)
    Xt, _, Mt = ws.features(ctx, te_warm, mu=mu, sigma=sd)
    it_w, st_w, _ = ws.solve(ctx, te_warm, net.predict(Xt, Mt))
    print("iters cold", it_c.mean(), "warm", it_w.mean(), flush=True)
    assert np.all(st_c == 0) and np.all(st_w == 0)
    assert it_w.mean() < 0.8 * it_c.mean()
    # same minima (the optimiser decides where it ends; a different local minimum would show here)
    Ec, Ew = host(te_cold.energy), host(te_warm.energy)
    assert np.mean(np.abs(Ec - Ew) < 1e-9 * np.abs(Ec)) >= 0.9
    # the trained network saved and loaded again predicts the same bits; a file
    # of another layout is refused
    import os
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "warm.npz")
        net.save(path, mu=mu, sigma=sd)
        net2 = ws.WarmStartMLP.load(ctx, path)
        assert net2.step == net.step
        Xt2, _, Mt2 = ws.features(ctx, rif.OnSet(ctx, test), mu=net2.mu, sigma=net2.sigma)
        assert np.array_equal(host(net2.predict(Xt2, Mt2)), host(net.predict(Xt, Mt)))
        bad = os.path.join(d, "bad.npz")
        np.savez(bad, layers=np.array([39, 64, 7]), theta=np.zeros(3, np.float32))
        with pytest.raises(ValueError):
            ws.WarmStartMLP.load(ctx, bad)
