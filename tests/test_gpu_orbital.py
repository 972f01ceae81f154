"""Orbital optimisation on the GPU (rif_orbital_step, rif_pnof_optimize)
against the FP64 oracle (oracle/orbital.py) and against two-electron full CI.

What is unique is compared: eigenvalues, the energy of every inner iteration,
and the orbitals up to the sign of each eigenvector.  Eigenvectors of a
degenerate eigenvalue are not unique (at the first step of an inner loop the
block outside Omega has a zero diagonal); those are checked for
orthonormality only, and the energy, which does not depend on them, is
compared at every iteration.
"""
import numpy as np
import pytest

import synth
from oracle import orbital as orb
from oracle import pnof7_ri as ri
from tests.gpu_util import host, to_dev

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


def sign_aligned(got, ref):
    """Flip each column of got to the sign of the matching column of ref."""
    s = np.sign(np.sum(got * ref, axis=0))
    s[s == 0] = 1
    return got * s


@pytest.mark.parametrize("shape", [(48, 192, 5, 1, 0), (37, 101, 3, 2, 11), (130, 259, 7, 3, 12)])
def test_orbital_step_matches_oracle(ctx, shape):
    import torch
    nb, na, npair, ncwo, seed = shape
    print("case orbital step", shape, flush=True)
    inst = synth.make_instance(nb, na, npair, ncwo, seed)
    t = to_dev(inst)
    out = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], npair, ncwo)
    lam = host(out["lam"])
    # distinct ascending diagonal: every eigenvector unique up to sign
    eps = np.sort(np.random.default_rng(seed).uniform(-5, 5, inst.n_mo))
    C_ref, w_ref = orb.orbital_step(inst.C, lam, eps)
    C = t["C"].clone()
    w = ctx.orbital_step(out["lam"], C, inst.occ.size, eps_in=torch.from_numpy(eps).cuda())
    ctx.sync()
    assert np.max(np.abs(host(w) - w_ref)) <= 1e-12 * np.max(np.abs(w_ref))
    Cg = sign_aligned(host(C), C_ref)
    assert np.max(np.abs(Cg - C_ref)) <= 1e-10
    assert np.allclose(host(C).T @ host(C), np.eye(inst.n_mo), atol=1e-12)


def test_inner_loop_matches_oracle(ctx):
    """30 inner iterations (first step from lambda_pp, then the eigenvalues)."""
    import torch
    inst = synth.workload("tiny")
    W = inst.occ.size
    print("case inner loop tiny 30 iterations", flush=True)
    ref = orb.inner_loop(inst.b, inst.C, inst.H, inst.occ, inst.pair_of, inst.n_pairs, 30, 1e-14)
    t = to_dev(inst)
    C = t["C"].clone()
    eps = torch.empty(inst.n_mo, dtype=torch.float64, device="cuda")
    out = None
    for it in range(30):
        out = ctx.build(t["b"], C, t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, out=out)
        ctx.sync()
        e = float(host(out["energy"])[0])
        assert abs(e - ref["energies"][it]) <= 1e-10 * abs(ref["energies"][it]), (it, e, ref["energies"][it])
        ctx.orbital_step(out["lam"], C, W, eps_in=eps if it else None, eps_out=eps)
    ctx.sync()
    Cg = host(C)
    assert np.allclose(Cg.T @ Cg, np.eye(inst.n_mo), atol=1e-12)
    # the Omega orbitals of the final set: equal to the oracle's up to sign
    Cw = sign_aligned(Cg[:, :W], ref["C"][:, :W])
    assert np.max(np.abs(Cw - ref["C"][:, :W])) <= 1e-8


def test_orbital_step_full_size(ctx):
    """Cyclohexane-like workload (n_bf = n_mo = 348): five inner iterations,
    energies against the oracle's."""
    import torch
    inst = synth.workload("c6h12")
    print("case inner loop c6h12 5 iterations", flush=True)
    ref = orb.inner_loop(inst.b, inst.C, inst.H, inst.occ, inst.pair_of, inst.n_pairs, 5, 1e-14)
    t = to_dev(inst)
    C = t["C"].clone()
    eps = torch.empty(inst.n_mo, dtype=torch.float64, device="cuda")
    out = None
    for it in range(5):
        out = ctx.build(t["b"], C, t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, out=out)
        ctx.sync()
        e = float(host(out["energy"])[0])
        assert abs(e - ref["energies"][it]) <= 1e-10 * abs(ref["energies"][it]), (it, e, ref["energies"][it])
        ctx.orbital_step(out["lam"], C, inst.occ.size, eps_in=eps if it else None, eps_out=eps)
    ctx.sync()
    Cg = host(C)
    assert np.allclose(Cg.T @ Cg, np.eye(inst.n_mo), atol=1e-11)


def run_loop(ctx, inst, C0, occ0, **kw):
    import torch
    t = to_dev(inst, C=C0)
    occ = torch.from_numpy(np.ascontiguousarray(occ0)).cuda()
    gamma = torch.zeros(inst.n_pairs * inst.n_cwo, dtype=torch.float64, device="cuda")
    res, he, hg = ctx.optimize(t["b"], t["C"], t["H"], occ, gamma, t["pair_of"], inst.n_pairs, inst.n_cwo,
                               hist_len=100000, **kw)
    ctx.sync()
    return res, he, hg, host(t["C"]), host(occ)


def test_full_loop_converges_to_a_stationary_point(ctx):
    """Fig. 1 loop (n_bf=20, n_aux=40, 2 pairs, Ncwo=1; about 2e4 inner
    iterations); the oracle checks the GPU's final point (energy, gradient,
    ON optimality) and runs the same loop."""
    from oracle import on_opt
    inst = synth.make_instance(20, 40, 2, 1, 31)
    print("case full loop n_bf=20 n_aux=40 pairs=2 ncwo=1 seed=31", flush=True)
    kw = dict(max_outer=40, max_inner=4000, tol_grad=1e-6, tol_energy=1e-9, on_tol=1e-10)
    res, he, hg, C, occ = run_loop(ctx, inst, inst.C, inst.occ, **kw)
    print("gpu loop", res, flush=True)
    assert res["status"] == 0 and res["on_status"] == 0
    assert np.allclose(C.T @ C, np.eye(inst.n_mo), atol=1e-11)
    # the oracle at the GPU's final point
    r = ri.build(inst.b, C, inst.H, occ, inst.pair_of, inst.n_pairs)
    assert abs(r["energy"] - res["energy"]) <= 1e-10 * abs(r["energy"])
    assert np.max(np.abs(r["grad"])) <= 1e-6 * 1.01
    # the ONs were optimised at the orbitals the last inner loop started from;
    # the energy change that loop made is below tol_energy, so they are close
    # to, not exactly at, the ON optimum of the final orbitals
    gam = on_opt.n_to_gamma(occ, inst.pair_of, inst.n_pairs, inst.n_cwo)
    g_on = on_opt.grad_gamma(gam, r["Hpp"], r["J"], r["K"], inst.pair_of, inst.n_pairs, inst.n_cwo)
    assert np.max(np.abs(g_on)) <= 1e-4
    assert len(he) == res["inner_total"] and he[-1] == res["energy"]
    # the oracle's own loop from the same start reaches the same energy
    ref = orb.outer_loop(inst.b, inst.C, inst.H, inst.occ, inst.pair_of, inst.n_pairs, inst.n_cwo,
                         kw["max_outer"], kw["max_inner"], kw["tol_grad"], kw["tol_energy"], kw["on_tol"])
    print("oracle loop", ref["energies"][-1], len(ref["energies"]), sum(ref["inner"]), flush=True)
    assert ref["converged"]
    assert abs(ref["energies"][-1] - res["energy"]) <= 1e-8 * abs(res["energy"])
    assert res["outer"] == len(ref["energies"])


def test_loop_reports_when_it_does_not_converge(ctx):
    """A mid-size molecule (n_bf=60, n_aux=150, 4 pairs, Ncwo=2) with a gradient
    tolerance the plain iteration does not reach within its limits: the loop
    returns status 1 (iteration limit), with every inner iteration recorded, a
    finite energy and max|G| above the tolerance, and orbitals still
    orthonormal."""
    inst = synth.make_instance(60, 150, 4, 2, 33)
    print("case loop not converging n_bf=60 n_aux=150 pairs=4 ncwo=2 seed=33", flush=True)
    kw = dict(max_outer=2, max_inner=40, tol_grad=1e-10, tol_energy=1e-12, on_tol=1e-10)
    res, he, hg, C, occ = run_loop(ctx, inst, inst.C, inst.occ, **kw)
    print("gpu loop", res, flush=True)
    assert res["status"] == 1
    assert res["outer"] == 2 and res["inner_total"] == 80 and len(he) == 80
    assert np.isfinite(res["energy"]) and res["max_grad"] > kw["tol_grad"]
    assert he[-1] == res["energy"] and hg[-1] == res["max_grad"]
    assert np.allclose(C.T @ C, np.eye(inst.n_mo), atol=1e-11)


def fci_two_electrons(h, eri):
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


@pytest.mark.parametrize("seed,direct", [(103, True), (104, True), (103, False)])
def test_full_loop_holds_two_electron_full_ci(ctx, seed, direct):
    """One pair over all 5 orbitals, started at the FCI natural orbitals and
    ONs: the GPU loop stays at the full-CI energy (inner builds with and
    without the per-MO AO matrices)."""
    nb = 5
    inst = synth.make_instance(nb, 3 * nb, 1, nb - 1, seed)
    print("case two-electron FCI seed", seed, flush=True)
    h = inst.C.T @ inst.H @ inst.C
    bm = np.einsum("mp,lmn,nq->lpq", inst.C, inst.b, inst.C)
    e_fci, X = fci_two_electrons(h, np.einsum("lpq,lrs->pqrs", bm, bm))
    c, U = np.linalg.eigh(X)
    order = np.argsort(-np.abs(c))
    c, U = c[order], U[:, order]
    c = c if c[0] > 0 else -c
    assert np.all(c[1:] < 0)
    occ0 = c ** 2
    occ0[0] = 1.0 - np.sum(occ0[1:])
    res, he, hg, C, occ = run_loop(ctx, inst, np.ascontiguousarray(inst.C @ U), occ0, max_outer=5,
                                   max_inner=50, tol_grad=1e-8, tol_energy=1e-11, on_tol=1e-10, direct=direct)
    print("gpu loop", res, "fci", e_fci, flush=True)
    assert res["status"] == 0
    assert abs(res["energy"] - e_fci) <= 1e-11 * abs(e_fci)
    assert min(he) >= e_fci - 1e-11 * abs(e_fci)


@pytest.mark.parametrize("mode,prec", [("bf16x6", 3), ("fp16x3", 4)])
def test_loop_in_split_precision(ctx, mode, prec):
    """The Fig. 1 loop with split-BF16x6 or split-FP16x3 builds (n_bf=20,
    n_aux=40) converges to max|G| <= 1e-5 at an energy within 1 uEh of the
    FP64 loop's."""
    inst = synth.make_instance(20, 40, 2, 1, 31)
    kw = dict(max_outer=40, max_inner=4000, tol_grad=1e-5, tol_energy=1e-9, on_tol=1e-10)
    r64, _, _, _, _ = run_loop(ctx, inst, inst.C, inst.occ, **kw)
    r6, _, _, _, _ = run_loop(ctx, inst, inst.C, inst.occ, prec=prec, **kw)
    print("fp64", r64, mode, r6, flush=True)
    assert r64["status"] == 0 and r6["status"] == 0
    assert abs(r6["energy"] - r64["energy"]) < 1e-6


def test_entry_point_argument_errors(ctx):
    """Bad arguments are refused with RIF_EINVAL before any launch."""
    import ctypes
    import torch
    import paper_2012_15662_amd as rif
    inst = synth.make_instance(10, 20, 2, 1, 40)
    t = to_dev(inst)
    occ = t["occ"].clone()
    gamma = torch.zeros(2, dtype=torch.float64, device="cuda")
    for bad in (dict(max_outer=0), dict(max_inner=0), dict(tol_grad=0.0), dict(on_tol=-1.0), dict(init_gamma=2)):
        with pytest.raises(rif.RifError) as e:
            ctx.optimize(t["b"], t["C"].clone(), t["H"], occ, gamma, t["pair_of"], inst.n_pairs, inst.n_cwo, **bad)
        assert e.value.status == -1, bad
    lam = torch.zeros((inst.n_mo, inst.occ.size), dtype=torch.float64, device="cuda")
    # n_omega > n_mo
    assert ctx.lib.rif_orbital_step(ctx.h, 10, 10, 11, ctypes.c_void_p(lam.data_ptr()), None,
                                    ctypes.c_void_p(t["C"].data_ptr()), ctypes.c_void_p(lam.data_ptr()), None) == -1
    # NULL b for the b preparation, FP64 pre-split
    assert ctx.lib.rif_prepare_b(ctx.h, 4, 4, None, None, 0.0, None, None, None, None, None) == -1
    assert ctx.lib.rif_presplit_b(ctx.h, 4, 4, ctypes.c_void_p(t["b"].data_ptr()), rif.FP64,
                                  ctypes.c_void_p(t["b"].data_ptr())) == -4
    ctx.sync()
