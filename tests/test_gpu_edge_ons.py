"""Occupation numbers at the edges of their range, through the C ABI.

* Hartree-Fock limit: every strong ON 1, every weak ON 0.  Every Phi_p and
  every intra-pair sqrt(n_q n_p) with a weak orbital vanishes, so the
  coefficient kernels meet exact zeros (and sqrt(0)).
* The bounds of the gamma map, n_g = 1/2 (gamma_g = pi/2) and n_g = 1
  (gamma_g = 0), mixed with interior pairs.

The full build (rif_build) and the build without per-MO AO matrices
(rif_build_direct) are compared with the FP64 oracle element by element at
1e-10 (normwise).  In the Hartree-Fock limit the GPU energy and gradient are
also compared with the closed-shell RHF energy tr D(H + F) and G_ai = 4 F_ai
built from the explicit four-index integrals (an independent route).
The ON optimiser started on the bounds must return finite results at the
oracle's energy of the ONs it reports.
"""
import math

import numpy as np
import pytest

import synth
from oracle import brute
from oracle import on_opt as oon
from oracle import pnof7_ri as ri
from tests.gpu_util import host, relerr, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-10
KEYS = ("b_half", "b_mo", "d", "J", "K", "lam", "grad")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    c = rif.Context()
    yield c
    c.close()


def with_strong(inst, strong):
    """Set pair g's strong ON to strong[g]; its weak orbitals share the rest."""
    occ = np.zeros(inst.n_omega)
    occ[:inst.n_pairs] = strong
    for p in range(inst.n_pairs, inst.n_omega):
        occ[p] = (1.0 - strong[inst.pair_of[p]]) / inst.n_cwo
    inst.occ = occ
    return inst


CASES = {
    "hf": lambda npair: np.ones(npair),
    "half": lambda npair: np.full(npair, 0.5),
    "mixed": lambda npair: np.array([(1.0, 0.5, 0.93)[g % 3] for g in range(npair)]),
}


def check(ctx, inst, direct):
    t = to_dev(inst)
    build = ctx.build_direct if direct else ctx.build
    out = build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    ctx.sync()
    ref = ri.build_instance(inst)
    errs = {k: relerr(host(out[k]), ref[k]) for k in KEYS + (() if direct else ("Jn", "Kn"))}
    e = float(host(out["energy"])[0])
    errs["energy"] = abs(e - ref["energy"]) / abs(ref["energy"])
    print(" ".join(f"{k}={v:.1e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v < TOL, (k, v)
    g = host(out["grad"])
    assert np.all(np.isfinite(g)) and np.array_equal(g, -g.T)
    return e, g


@pytest.mark.parametrize("direct", [False, True])
@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("shape", [(40, 110, 4, 2, 71), (130, 259, 7, 3, 72)])
def test_edge_ons_match_oracle(ctx, shape, case, direct):
    nb, na, npair, ncwo, seed = shape
    print(f"case {case} direct={direct} n_bf={nb} n_aux={na} pairs={npair} ncwo={ncwo} seed={seed}", flush=True)
    check(ctx, with_strong(synth.make_instance(nb, na, npair, ncwo, seed), CASES[case](npair)), direct)


@pytest.mark.parametrize("direct", [False, True])
def test_hf_limit_against_rhf(ctx, direct):
    """Closed-shell RHF from the explicit (mu nu|sigma lambda) = sum_l b b."""
    inst = with_strong(synth.make_instance(24, 60, 3, 2, 73), np.ones(3))
    print(f"case hf-vs-rhf direct={direct}", flush=True)
    e, g = check(ctx, inst, direct)
    eri = brute.eri4(inst.b)
    E_hf, F = brute.rhf(eri, inst.H, inst.C[:, :inst.n_pairs])
    assert abs(e - E_hf) < 1e-10 * abs(E_hf)
    F_mo = inst.C.T @ F @ inst.C
    no = inst.n_pairs
    # G_ai = 4 F_ai between virtual a and occupied i; zero within each block
    assert np.max(np.abs(g[no:, :no] - 4.0 * F_mo[no:, :no])) < 1e-10 * np.max(np.abs(F_mo))
    assert np.max(np.abs(g[:no, :no])) < 1e-12 and np.max(np.abs(g[no:, no:])) < 1e-12


@pytest.mark.parametrize("where", ["hf", "half"])
def test_on_optimizer_started_on_the_bounds(ctx, where):
    """gamma_g = 0 (n_g = 1) or pi/2 (n_g = 1/2) for every pair, the weak
    angles at 0 (all weak ON on the first weak orbital)."""
    import paper_2012_15662_amd as rif
    inst = synth.make_instance(30, 90, 3, 2, 74)
    o = ri.build_instance(inst)
    dev = lambda a: __import__("torch").from_numpy(np.ascontiguousarray(a)).cuda()
    prob = (dev(o["Hpp"]), dev(o["J"]), dev(o["K"]), dev(inst.pair_of.astype(np.int32)), inst.n_pairs,
            inst.n_cwo)
    onset = rif.OnSet(ctx, [prob], tol=1e-8)
    g0 = np.zeros(inst.n_pairs * inst.n_cwo)
    if where == "half":
        g0[::inst.n_cwo] = math.pi / 2
    onset.gamma.copy_(dev(g0))
    print(f"case on-optimizer start={where}", flush=True)
    ctx.on_optimize(onset)
    ctx.sync()
    st, it = int(host(onset.status)[0]), int(host(onset.iters)[0])
    E = float(host(onset.energy)[0])
    gam = host(onset.gamma)
    n = host(onset.occ)
    print(f"status={st} iters={it} E={E:.12f}", flush=True)
    assert st in (0, 1) and np.isfinite(E) and np.all(np.isfinite(gam)) and np.all(np.isfinite(n))
    # the reported ONs are the map of the reported gamma, and E is their energy
    n_ref = oon.gamma_to_n(gam, inst.pair_of, inst.n_pairs, inst.n_cwo)
    assert np.max(np.abs(n - n_ref)) < 1e-14
    E_ref = oon.energy_gamma(gam, o["Hpp"], o["J"], o["K"], inst.pair_of, inst.n_pairs, inst.n_cwo)
    assert abs(E - E_ref) < 1e-12 * abs(E_ref)
    if st == 0:
        gr = oon.grad_gamma(gam, o["Hpp"], o["J"], o["K"], inst.pair_of, inst.n_pairs, inst.n_cwo)
        assert np.max(np.abs(gr)) <= 1e-7
