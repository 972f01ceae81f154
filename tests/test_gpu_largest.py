"""Parity at the largest workload: n_bf=1000, n_aux=3000, 60 pairs, Ncwo=6
(n_omega=420, n_mo=1000; b is 24 GB in FP64).

b is drawn on the GPU by the seeded input generator and copied to the host.
The FP64 oracle then builds every output on the host's cores. That takes about
9.3e12 flops of batched BLAS and about 90 GB of host memory.

The GPU side runs with autotuned tiles. Every element of b_half, b_mo, d, J, K,
Jn, Kn, lambda and G is compared, and so is the energy: FP64 to 1e-10 relative
(normwise for arrays). The direct gradient is held to the same bound. The
reduced-precision modes are compared on the energy and gradient only:
1 uEh and 1e-6 normwise for FP32 and BF16x6, 5 uEh and 1e-6 for FP16x3 (2.0 uEh
here), 1e-4 for BF16x3.  Builds that read b stored pre-split (FP16x3, BF16x6)
must equal the ones that split b on load, bitwise.
"""
import time

import numpy as np
import pytest

import synth
from oracle import pnof7_ri as ri
from tests.gpu_util import host, relerr

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
KEYS = ("b_half", "b_mo", "d", "J", "K", "Jn", "Kn", "lam", "grad")
SIZE = (1000, 3000, 60, 6)   # n_bf, n_aux, pairs, Ncwo
SEED = 31


@pytest.fixture(scope="module")
def case():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    print(f"case largest n_bf={SIZE[0]} n_aux={SIZE[1]} pairs={SIZE[2]} ncwo={SIZE[3]} seed={SEED}", flush=True)
    t, npair, ncwo = synth.make_instance_device(*SIZE, SEED)
    torch.cuda.synchronize()
    c = rif.Context()
    c.autotune(True)
    ts = time.perf_counter()
    b = host(t["b"])
    C, H, occ = host(t["C"]), host(t["H"]), host(t["occ"])
    pair_of = host(t["pair_of"]).astype(np.int64)
    print(f"inputs on the host in {time.perf_counter() - ts:.1f} s; oracle build ...", flush=True)
    ts = time.perf_counter()
    ref = ri.build(b, C, H, occ, pair_of, npair)
    del b
    print(f"oracle done in {time.perf_counter() - ts:.1f} s, E={ref['energy']:.12f}", flush=True)
    yield c, t, npair, ncwo, ref
    c.close()


def build_errors(c, t, npair, ncwo, ref, prec, keys=KEYS, direct=False):
    build = c.build_direct if direct else c.build
    out = build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], npair, ncwo, prec=prec)
    c.sync()
    e = {}
    for k in keys:
        e[k] = relerr(host(out[k]), ref[k])
    e["dE"] = abs(float(host(out["energy"])[0]) - ref["energy"])
    return e, out


def test_fp64_every_element(case):
    c, t, npair, ncwo, ref = case
    e, out = build_errors(c, t, npair, ncwo, ref, 0)
    print("fp64 largest", " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    for k in KEYS:
        assert e[k] < 1e-10, (k, e[k])
    assert e["dE"] / abs(ref["energy"]) < 1e-10
    Kn = host(out["Kn"])
    assert np.array_equal(Kn, Kn.transpose(0, 2, 1))


def test_direct_gradient(case):
    c, t, npair, ncwo, ref = case
    e, _ = build_errors(c, t, npair, ncwo, ref, 0, keys=("lam", "grad"), direct=True)
    print("direct largest", " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    assert e["lam"] < 1e-10 and e["grad"] < 1e-10
    assert e["dE"] / abs(ref["energy"]) < 1e-10


@pytest.mark.parametrize("mode,prec,tol_e,tol_g", [
    ("fp32", 1, 1e-6, 1e-6),
    ("bf16x6", 3, 1e-6, 1e-6),
])
def test_reduced_precision(case, mode, prec, tol_e, tol_g):
    """The modes that meet the reduced-precision target at this size."""
    c, t, npair, ncwo, ref = case
    e, _ = build_errors(c, t, npair, ncwo, ref, prec, keys=("J", "K", "grad"))
    print(mode, "largest", " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    assert e["dE"] < tol_e and e["grad"] < tol_g


@pytest.mark.parametrize("mode,prec,bound_e,bound_g", [
    ("bf16x3", 2, 1e-4, 1e-4),
    ("fp16x3", 4, 1e-5, 1e-6),   # about 2 uEh: the f16 MFMA's summation width
])
def test_documented_miss(case, mode, prec, bound_e, bound_g):
    """Modes that do not meet 1 uEh at this size: only their miss is bounded."""
    c, t, npair, ncwo, ref = case
    e, _ = build_errors(c, t, npair, ncwo, ref, prec, keys=("J", "K", "grad"))
    print(mode, "largest (documented miss)", " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    assert e["dE"] < bound_e and e["grad"] < bound_g


@pytest.mark.parametrize("mode,prec", [("fp16x3", 4), ("bf16x6", 3)])
def test_presplit_bitwise_at_largest_size(case, mode, prec):
    """b stored pre-split (24 or 36 GB of piece planes here, rows of 3e6 and
    1e6 with 64-bit offsets) gives bitwise the build that splits b on load."""
    import torch
    c, t, npair, ncwo, ref = case
    bs = c.presplit_b(t["b"], prec)
    a = c.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], npair, ncwo, prec=prec)
    b = c.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], npair, ncwo, prec=prec, b_split=bs)
    c.sync()
    for k in ("b_half", "Jn", "Kn", "energy", "lam", "grad"):
        assert torch.equal(a[k], b[k]), k
    print(mode, "largest: pre-split build bitwise equal", flush=True)
    del bs, a, b
    torch.cuda.empty_cache()
