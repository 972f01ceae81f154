"""Full-size parity at the cyclodecane-like workload (n_bf=580, n_aux=1740, 40
pairs, Ncwo=4, n_mo=580): the same instance bench.py times, built on the GPU
with autotuned tiles (the launch configuration the bench uses), every output
element compared with the FP64 oracle.

FP64 is held to 1e-10 relative (normwise for arrays); FP32 and split BF16x6,
which meet the reduced-precision target here, to 1 uEh in the energy and 1e-6
normwise in the gradient.  Two modes are documented misses of that target at
this size and are not claimed to meet it: split FP16x3 (about 1.1 uEh; the
f16 MFMA keeps about 24 bits of each group of eight products, and 11-bit high
pieces give 22-bit products, so the smaller products of a group lose bits)
and BF16x3 (two 8-bit pieces, about 17 uEh).  Their tests only bound the miss
(5 uEh and 1e-4) so that a regression still fails, and print the errors.
"""
import numpy as np
import pytest

import synth
from oracle import pnof7_ri as ri
from tests.gpu_util import host, relerr, to_dev

pytestmark = pytest.mark.gpu
KEYS = ("b_half", "b_mo", "d", "J", "K", "Jn", "Kn", "lam", "grad")


@pytest.fixture(scope="module")
def case():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    print("case cyclodecane-like n_bf=580 n_aux=1740 pairs=40 ncwo=4 (bench workload c10h20)", flush=True)
    inst = synth.workload("c10h20")
    ref = ri.build_instance(inst)
    c = rif.Context()
    c.autotune(True)
    t = to_dev(inst)
    inst.b = None   # the oracle is done with the host copy
    yield c, t, inst, ref
    c.close()


def build_errors(c, t, inst, ref, prec):
    out = c.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec)
    c.sync()
    e = {k: relerr(host(out[k]), ref[k]) for k in KEYS}
    e["dE"] = abs(float(host(out["energy"])[0]) - ref["energy"])
    return e, out


def test_fp64_every_element(case):
    c, t, inst, ref = case
    e, out = build_errors(c, t, inst, ref, 0)
    print("fp64", " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    for k in KEYS:
        assert e[k] < 1e-10, (k, e[k])
    assert e["dE"] / abs(ref["energy"]) < 1e-10
    Jn, Kn = host(out["Jn"]), host(out["Kn"])
    assert np.array_equal(Jn, Jn.transpose(0, 2, 1)) and np.array_equal(Kn, Kn.transpose(0, 2, 1))


@pytest.mark.parametrize("mode,prec,tol_e,tol_g", [
    ("fp32", 1, 1e-6, 1e-6),
    ("bf16x6", 3, 1e-6, 1e-6),
])
def test_reduced_precision(case, mode, prec, tol_e, tol_g):
    c, t, inst, ref = case
    e, _ = build_errors(c, t, inst, ref, prec)
    print(mode, "c10h20", " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    assert e["dE"] < tol_e and e["grad"] < tol_g


@pytest.mark.parametrize("mode,prec,bound_e,bound_g", [
    ("bf16x3", 2, 1e-4, 1e-4),
    ("fp16x3", 4, 5e-6, 1e-6),
])
def test_documented_miss(case, mode, prec, bound_e, bound_g):
    """Modes that do not meet 1 uEh at this size: only their miss is bounded."""
    c, t, inst, ref = case
    e, _ = build_errors(c, t, inst, ref, prec)
    print(mode, "c10h20 (documented miss)", " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    assert e["dE"] < bound_e and e["grad"] < bound_g
