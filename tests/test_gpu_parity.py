"""FP64 HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerance: the FP64 path must match the oracle to 1e-10 relative (normwise:
max|diff| / max|ref| for arrays, |diff|/|ref| for the energy).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import pnof7_ri as ri
from tests.gpu_util import host, relerr, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    c = rif.Context()
    yield c
    c.close()


def run_and_compare(ctx, inst, C=None, functional="pnof7"):
    import paper_2012_15662_amd as rif
    print(f"case n_bf={inst.n_bf} n_aux={inst.n_aux} pairs={inst.n_pairs} ncwo={inst.n_cwo} "
          f"n_mo={inst.n_mo} seed={inst.seed}", flush=True)
    t = to_dev(inst, C)
    fn = rif.PNOF7 if functional == "pnof7" else rif.PNOF5
    out = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo,
                    functional=fn)
    ctx.sync()
    ref = ri.build(inst.b, inst.C if C is None else C, inst.H, inst.occ, inst.pair_of,
                   inst.n_pairs, functional)
    errs = {k: relerr(host(out[k]), ref[k]) for k in ("b_half", "b_mo", "d", "J", "K", "Jn", "Kn",
                                                      "lam", "grad")}
    errs["energy"] = abs(float(host(out["energy"])[0]) - ref["energy"]) / abs(ref["energy"])
    print(" ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v < TOL, (k, v)
    # exact symmetry of the per-MO AO matrices (mirrored writes)
    Jn, Kn = host(out["Jn"]), host(out["Kn"])
    assert np.array_equal(Jn, Jn.transpose(0, 2, 1))
    assert np.array_equal(Kn, Kn.transpose(0, 2, 1))
    return out, ref


@pytest.mark.parametrize("shape", [
    (48, 192, 5, 1, 0),      # tiny workload
    (37, 101, 3, 2, 11),     # ragged everything
    (130, 259, 7, 3, 12),    # more than one 128-tile in n_bf, ragged tails
    (4, 1, 1, 1, 13),        # n_aux = 1, n_omega = 2
    (16, 16, 8, 1, 14),      # n_omega = n_bf = n_mo
    (200, 67, 13, 4, 15),    # n_omega = 65 (> 64, ragged), n_aux < n_bf
])
def test_build_matches_oracle(ctx, shape):
    nb, na, npair, ncwo, seed = shape
    run_and_compare(ctx, synth.make_instance(nb, na, npair, ncwo, seed))


def test_n_mo_smaller_than_n_bf(ctx):
    run_and_compare(ctx, synth.make_instance(50, 90, 4, 2, 16, n_mo=30))


def test_pnof5(ctx):
    run_and_compare(ctx, synth.make_instance(40, 80, 3, 2, 17), functional="pnof5")


def test_explicit_nondefault_pair_map(ctx):
    import torch
    import paper_2012_15662_amd as rif
    inst = synth.make_instance(36, 70, 3, 2, 18)
    rng = np.random.default_rng(0)
    weak = rng.permutation(np.arange(inst.n_pairs, inst.n_omega))
    pm = inst.pair_of.copy()
    for i, w in enumerate(weak):
        pm[w] = i % inst.n_pairs
    occ = inst.occ.copy()
    for g in range(inst.n_pairs):
        occ[(pm == g) & (np.arange(inst.n_omega) >= inst.n_pairs)] = (1 - occ[g]) / inst.n_cwo
    inst.pair_of, inst.occ = pm.astype(np.int32), occ
    run_and_compare(ctx, inst)


def test_default_pair_map_when_null(ctx):
    import torch
    import paper_2012_15662_amd as rif
    inst = synth.make_instance(30, 60, 3, 2, 19)
    t = to_dev(inst)
    o1 = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    e1, g1 = host(o1["energy"]).copy(), host(o1["grad"]).copy()
    o2 = ctx.build(t["b"], t["C"], t["H"], t["occ"], None, inst.n_pairs, inst.n_cwo)
    ctx.sync()
    assert np.array_equal(e1, host(o2["energy"])) and np.array_equal(g1, host(o2["grad"]))


def test_cyclohexane_like_full_size(ctx):
    """n_bf=348, n_aux=1044, 24 pairs, Ncwo=4 with a rotated C, every element."""
    inst = synth.workload("c6h12")
    Cs = synth.rotation_sequence(inst.C, 3)
    run_and_compare(ctx, inst, C=Cs[2])


def test_deterministic_bitwise(ctx):
    inst = synth.make_instance(150, 300, 10, 3, 21)
    t = to_dev(inst)
    o1 = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    a = {k: host(v).copy() for k, v in o1.items()}
    o2 = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    ctx.sync()
    for k, v in o2.items():
        assert np.array_equal(a[k], host(v)), k


@pytest.mark.parametrize("prec", [0, 3])
def test_build_equals_the_four_abi_steps(ctx, prec):
    """rif_build (two streams) and the four step calls (one stream) run the same
    kernels in the same reduction orders: identical results, bit for bit."""
    inst = synth.make_instance(139, 157, 9, 3, 24)
    t = to_dev(inst)
    args = (t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    o1 = ctx.build(*args, prec=prec)
    a = {k: host(v).copy() for k, v in o1.items()}
    o2 = ctx.build_steps(*args, prec=prec)
    ctx.sync()
    for k, v in o2.items():
        assert np.array_equal(a[k], host(v)), k


def test_invalid_occupations_reported(ctx):
    import torch
    import paper_2012_15662_amd as rif
    inst = synth.make_instance(20, 40, 2, 1, 22)
    t = to_dev(inst)
    t["occ"][0] += 0.01   # pair 0 no longer sums to 1
    ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    with pytest.raises(rif.RifError) as e:
        ctx.sync()
    assert e.value.status == -1 and "sum to 1" in str(e.value)
    ctx.sync()   # cleared


def test_shape_and_pointer_errors(ctx):
    import ctypes
    import torch
    import paper_2012_15662_amd as rif
    lib = ctx.lib
    buf = torch.zeros(64, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    # n_omega > n_mo
    assert lib.rif_transform(ctx.h, 4, 4, 5, 4, p, p, rif.FP64, p, p, p) == -1
    # NULL output
    assert lib.rif_transform(ctx.h, 4, 4, 2, 4, p, p, rif.FP64, None, p, p) == -1
    assert b"NULL" in lib.rif_last_error(ctx.h)
    # n_omega != pairs (1 + ncwo) > n_mo
    assert lib.pnof7_energy_grad(ctx.h, 4, 4, 2, 2, None, p, p, p, p, p, p, p, rif.FP64, p, p, p) == -1
    assert lib.rif_jk_mo(ctx.h, 0, 3, p, p, rif.FP64, p, p) == -1
    assert lib.rif_jk_ao_per_mo(ctx.h, 4, 4, 5, p, p, p, rif.FP64, p, p) == -1
    assert lib.rif_transform(None, 4, 4, 2, 4, p, p, rif.FP64, p, p, p) == -1


def test_workspace_limit(ctx):
    import paper_2012_15662_amd as rif
    c2 = rif.Context()
    c2.set_workspace_limit(1024)
    inst = synth.make_instance(64, 300, 4, 2, 23)
    t = to_dev(inst)
    with pytest.raises(rif.RifError) as e:
        c2.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    assert e.value.status == -2
    c2.close()


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_every_tile_variant(ctx, variant):
    """Each tile shape of every MFMA kernel, on a case with ragged tails in all dims."""
    ctx.set_tile_variant(variant)
    try:
        run_and_compare(ctx, synth.make_instance(139, 157, 9, 3, 30 + variant))
    finally:
        ctx.set_tile_variant(-1)


def test_autotune_picks_and_matches(ctx):
    import paper_2012_15662_amd as rif
    c2 = rif.Context()
    c2.autotune(True)
    inst = synth.make_instance(101, 230, 6, 4, 40)
    t = to_dev(inst)
    o = c2.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    c2.sync()
    rep = c2.tune_report()
    for k in ("half_transform", "mo_transform", "jao", "kao", "fock"):
        assert k in rep, rep
    ref = ri.build_instance(inst)
    assert relerr(host(o["grad"]), ref["grad"]) < TOL
    assert abs(float(host(o["energy"])[0]) - ref["energy"]) < TOL * abs(ref["energy"])
    c2.close()


def test_profile_all_and_one_kernel(ctx):
    """Per-launch event timing: every kernel by default, one named kernel with
    rif_profile_only, and the results of the profiled builds unchanged."""
    inst = synth.make_instance(64, 150, 5, 2, 41)
    t = to_dev(inst)
    args = (t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    o0 = ctx.build(*args)
    ref = host(o0["grad"]).copy()
    try:
        ctx.profile(True)
        ctx.build(*args)
        ctx.build(*args)
        allk = ctx.profile_report()
        assert {"half_transform", "mo_transform", "jao", "kao", "fock"} <= set(allk), allk
        assert allk["half_transform"][0] == 2 and allk["kao"][0] == 2, allk
        ctx.profile(True, only="half_transform")
        for _ in range(3):
            o = ctx.build(*args)
        one = ctx.profile_report()
        assert set(one) == {"half_transform"}, one
        assert one["half_transform"][0] == 3 and one["half_transform"][1] > 0.0
        assert np.array_equal(host(o["grad"]), ref)
        ctx.profile(True, only="no_such_kernel")
        ctx.build(*args)
        assert ctx.profile_report() == {}
    finally:
        ctx.profile(False)
