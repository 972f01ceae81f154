"""rif_build_direct (energy, lambda and G without the per-MO AO matrices)
against the FP64 oracle, through the C ABI.

FP64: 1e-10 relative (normwise for arrays) on every output it writes, over the
same ragged and degenerate shapes as the rif_build tests and every tile
variant.  Reduced precision: 1 uEh in the energy and 1e-6 (normwise) in the
gradient for FP32 and split BF16x6; BF16x3 to 1e-4.  The energy of the two
entry points is the same computation, so it must agree bitwise.
"""
import numpy as np
import pytest

import synth
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


def direct_errors(ctx, inst, prec=0, functional="pnof7"):
    import paper_2012_15662_amd as rif
    print(f"case direct n_bf={inst.n_bf} n_aux={inst.n_aux} pairs={inst.n_pairs} ncwo={inst.n_cwo} "
          f"n_mo={inst.n_mo} seed={inst.seed} prec={prec} {functional}", flush=True)
    t = to_dev(inst)
    fn = rif.PNOF7 if functional == "pnof7" else rif.PNOF5
    out = ctx.build_direct(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo,
                           prec=prec, functional=fn)
    ctx.sync()
    ref = ri.build(inst.b, inst.C, inst.H, inst.occ, inst.pair_of, inst.n_pairs, functional)
    e = {k: relerr(host(out[k]), ref[k]) for k in KEYS}
    e["dE"] = abs(float(host(out["energy"])[0]) - ref["energy"])
    e["energy"] = e["dE"] / abs(ref["energy"])
    print(" ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    return e, out, t


@pytest.mark.parametrize("shape", [
    (48, 192, 5, 1, 0),      # tiny workload
    (37, 101, 3, 2, 11),     # ragged everything
    (130, 259, 7, 3, 12),    # more than one 128-tile in n_bf, ragged tails
    (4, 1, 1, 1, 13),        # n_aux = 1, n_omega = 2
    (16, 16, 8, 1, 14),      # n_omega = n_bf = n_mo
    (200, 67, 13, 4, 15),    # n_omega = 65, n_aux < n_bf
])
def test_direct_matches_oracle(ctx, shape):
    e, _, _ = direct_errors(ctx, synth.make_instance(*shape))
    for k in KEYS + ("energy",):
        assert e[k] < TOL, (k, e[k])


def test_direct_fewer_mos_and_pnof5(ctx):
    e, _, _ = direct_errors(ctx, synth.make_instance(50, 90, 4, 2, 16, n_mo=30))
    assert max(e[k] for k in KEYS + ("energy",)) < TOL
    e, _, _ = direct_errors(ctx, synth.make_instance(40, 80, 3, 2, 17), functional="pnof5")
    assert max(e[k] for k in KEYS + ("energy",)) < TOL


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_direct_every_tile_variant(ctx, variant):
    ctx.set_tile_variant(variant)
    try:
        e, _, _ = direct_errors(ctx, synth.make_instance(139, 157, 9, 3, 30 + variant))
    finally:
        ctx.set_tile_variant(-1)
    assert max(e[k] for k in KEYS + ("energy",)) < TOL


def test_direct_agrees_with_build(ctx):
    inst = synth.make_instance(101, 230, 6, 4, 40)
    e, out, t = direct_errors(ctx, inst)
    full = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    ctx.sync()
    assert np.array_equal(host(full["energy"]), host(out["energy"]))
    assert np.array_equal(host(full["J"]), host(out["J"])) and np.array_equal(host(full["K"]), host(out["K"]))
    assert relerr(host(out["grad"]), host(full["grad"])) < 1e-12


@pytest.mark.parametrize("mode,prec,tol_e,tol_g", [
    ("fp32", 1, 1e-6, 1e-6),
    ("bf16x6", 3, 1e-6, 1e-6),
    ("bf16x3", 2, 1e-4, 1e-4),
    ("fp16x3", 4, 1e-6, 1e-6),
])
def test_direct_reduced_precision_full_size(ctx, mode, prec, tol_e, tol_g):
    """Cyclohexane-like workload (n_bf=348, n_aux=1044, 24 pairs, Ncwo=4)."""
    e, _, _ = direct_errors(ctx, synth.workload("c6h12"), prec=prec)
    print(mode, "dE", e["dE"], "grad", e["grad"], flush=True)
    assert e["dE"] < tol_e and e["grad"] < tol_g


def test_direct_fp64_full_size(ctx):
    e, _, _ = direct_errors(ctx, synth.workload("c6h12"))
    assert max(e[k] for k in KEYS + ("energy",)) < TOL
