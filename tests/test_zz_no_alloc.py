"""rif_jk_mo_noalloc (the entry point that allocates nothing) against
rif_jk_mo through the C ABI: bitwise-equal J and K on two calls in a row, the
second on a smaller input, in FP64 and a reduced mode; the size limit is
refused with RIF_ENOMEM."""
import numpy as np
import pytest

import synth
from oracle import pnof7_ri as ri
from tests.gpu_util import host, relerr, to_dev

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


def jk_inputs(ctx, shape, prec):
    nb, na, npair, ncwo, seed = shape
    inst = synth.make_instance(nb, na, npair, ncwo, seed)
    t = to_dev(inst)
    _, bmo, d = ctx.transform(t["b"], t["C"], inst.n_omega, prec)
    return inst, bmo, d


@pytest.mark.parametrize("prec", [0, 3])
def test_noalloc_equals_jk_mo_twice(ctx, prec):
    import torch
    for shape in [(130, 259, 7, 3, 81), (40, 90, 3, 2, 82)]:    # the second call is smaller
        print(f"case noalloc prec={prec} shape={shape}", flush=True)
        inst, bmo, d = jk_inputs(ctx, shape, prec)
        J0, K0 = ctx.jk_mo(bmo, d, prec)
        w = inst.n_omega
        J1 = torch.full((w, w), float("nan"), dtype=torch.float64, device="cuda")
        K1 = torch.full((w, w), float("nan"), dtype=torch.float64, device="cuda")
        ctx.jk_mo_noalloc(bmo, d, J1, K1, prec)
        ctx.sync()
        assert np.array_equal(host(J0), host(J1)) and np.array_equal(host(K0), host(K1))
        if prec == 0:
            ref = ri.build_instance(inst)
            assert relerr(host(J1), ref["J"]) < 1e-10 and relerr(host(K1), ref["K"]) < 1e-10


def test_noalloc_refuses_beyond_its_scratch(ctx):
    import torch
    import paper_2012_15662_amd as rif
    w = 1100                     # 2 * 1100^2 doubles > 16 MiB
    bmo = torch.zeros((1, w, w), dtype=torch.float64, device="cuda")
    d = torch.zeros((1, w), dtype=torch.float64, device="cuda")
    J = torch.empty((w, w), dtype=torch.float64, device="cuda")
    K = torch.empty((w, w), dtype=torch.float64, device="cuda")
    with pytest.raises(rif.RifError) as e:
        ctx.jk_mo_noalloc(bmo, d, J, K, 0)
    assert e.value.status == -2 and "scratch" in str(e.value)
