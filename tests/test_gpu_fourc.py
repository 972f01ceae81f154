"""The conventional four-centre path (Table 1, Eqs. (3)-(5)) on the GPU.

* Step 0 (rif_eri4_from_b): the packed integrals eri[(mu nu)][sigma][lambda]
  against the oracle's explicit (mu nu|sigma lambda) = sum_l b b, every element.
* Steps 1-3 (rif_jk_4c): J^q, K^q, J and K against the oracle's Table 1 route
  (brute.table1 on the explicit integrals) at small sizes, and against the RI
  oracle at larger ones: with integrals built from the same factors the two
  routes agree exactly (a CPU pin), so both compare with an oracle result.

FP64 throughout, held to 1e-10 (normwise).
"""
import numpy as np
import pytest

import synth
from oracle import brute
from oracle import pnof7_ri as ri
from tests.gpu_util import host, relerr

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


def run_4c(ctx, inst):
    import torch
    b = torch.from_numpy(inst.b).cuda()
    C = torch.from_numpy(inst.C).cuda()
    eri = ctx.eri4_from_b(b)
    out = ctx.jk_4c(eri, C, inst.n_omega)
    ctx.sync()
    return eri, out


@pytest.mark.parametrize("shape", [(12, 30, 2, 1, 91), (25, 40, 3, 2, 92), (33, 70, 4, 3, 93), (2, 1, 1, 1, 94)])
def test_four_centre_matches_table1(ctx, shape):
    nb, na, npair, ncwo, seed = shape
    print(f"case 4c n_bf={nb} n_aux={na} pairs={npair} ncwo={ncwo}", flush=True)
    inst = synth.make_instance(nb, na, npair, ncwo, seed)
    eri, out = run_4c(ctx, inst)
    ref4 = brute.eri4(inst.b)
    iu = np.triu_indices(nb)
    assert relerr(host(eri).reshape(-1, nb, nb), ref4[iu]) < TOL
    W = inst.n_omega
    J, K, Jq, Kq = brute.table1(ref4, inst.C[:, :W])
    for k, ref in (("Jn", Jq), ("Kn", Kq), ("J", J), ("K", K)):
        e = relerr(host(out[k]), ref)
        print(k, f"{e:.2e}", flush=True)
        assert e < TOL, (k, e)
    assert np.array_equal(host(out["Jn"]), host(out["Jn"]).transpose(0, 2, 1))
    assert np.array_equal(host(out["Kn"]), host(out["Kn"]).transpose(0, 2, 1))


@pytest.mark.parametrize("shape", [(130, 200, 7, 3, 95), (64, 192, 5, 2, 96)])
def test_four_centre_matches_ri_oracle(ctx, shape):
    nb, na, npair, ncwo, seed = shape
    print(f"case 4c-vs-RI n_bf={nb} n_aux={na} pairs={npair} ncwo={ncwo}", flush=True)
    inst = synth.make_instance(nb, na, npair, ncwo, seed)
    _, out = run_4c(ctx, inst)
    ref = ri.build_instance(inst)
    for k in ("Jn", "Kn", "J", "K"):
        e = relerr(host(out[k]), ref[k])
        print(k, f"{e:.2e}", flush=True)
        assert e < TOL, (k, e)


def test_four_centre_cyclohexane_size(ctx):
    """n_bf=348, n_omega=120: the integrals take 59 GB of HBM (first pair
    packed), Z 20 GB; J, K and sampled J^q/K^q rows against the RI oracle."""
    import torch
    inst = synth.workload("c6h12")
    print("case 4c cyclohexane-like n_bf=348 n_aux=1044 pairs=24 ncwo=4", flush=True)
    ref = ri.build_instance(inst)
    eri, out = run_4c(ctx, inst)
    for k in ("J", "K"):
        e = relerr(host(out[k]), ref[k])
        print(k, f"{e:.2e}", flush=True)
        assert e < TOL, (k, e)
    rng = np.random.default_rng(5)
    for q in rng.choice(inst.n_omega, 6, replace=False):
        for k in ("Jn", "Kn"):
            assert relerr(host(out[k][q]), ref[k][q]) < TOL, (k, q)
    del eri
    torch.cuda.empty_cache()


def test_four_centre_argument_errors(ctx):
    import torch
    import paper_2012_15662_amd as rif
    C = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    eri = torch.zeros(int(ctx.lib.rif_eri4_bytes(8)) // 8, dtype=torch.float64, device="cuda")
    with pytest.raises(rif.RifError) as e:
        ctx.jk_4c(eri, C, 9)             # n_omega > n_mo
    assert e.value.status == -1
