"""Batched builds of uneven molecules (grouped persistent launches, hipGraph).

Each molecule's result from the batch must equal the single-molecule build
with the same tile variant bit for bit, match the FP64 oracle to 1e-10, and
every replay of the captured graph -- with other GPU work and synchronisations
between replays -- must reproduce the eager result.
"""
import numpy as np
import pytest

import synth
from oracle import pnof7_ri as ri
from tests.gpu_util import host, relerr, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(120, 360, 10, 2, 50), (61, 183, 5, 2, 51), (37, 111, 3, 2, 52), (150, 450, 12, 2, 53),
          (64, 192, 5, 2, 54), (90, 270, 7, 2, 55)]
KEYS = ("b_half", "b_mo", "d", "J", "K", "Jn", "Kn", "energy", "lam", "grad")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    c = rif.Context()
    yield c
    c.close()


def make_items(prec):
    insts = [synth.make_instance(*s) for s in SHAPES]
    return insts, [(to_dev(i), i.n_pairs, i.n_cwo, None) for i in insts]


@pytest.mark.parametrize("variant", [0, 1])
def test_batch_equals_single_and_oracle(ctx, variant):
    import paper_2012_15662_amd as rif
    ctx.set_tile_variant(variant)
    try:
        insts, items = make_items(rif.FP64)
        batch = ctx.batch(items)
        batch.run(use_graph=False)
        ctx.sync()
        for inst, (inp, npair, ncwo, _), out in zip(insts, items, batch.outs):
            print(f"case n_bf={inst.n_bf} n_aux={inst.n_aux} pairs={npair}", flush=True)
            single = ctx.build_instance(inp, npair, ncwo)
            ctx.sync()
            for k in KEYS:
                assert np.array_equal(host(out[k]), host(single[k])), k
            ref = ri.build_instance(inst)
            assert abs(float(host(out["energy"])[0]) - ref["energy"]) < 1e-10 * abs(ref["energy"])
            for k in ("J", "K", "Jn", "Kn", "grad"):
                assert relerr(host(out[k]), ref[k]) < 1e-10, k
        batch.close()
    finally:
        ctx.set_tile_variant(-1)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_fp32_batch_equals_single(ctx, variant):
    """FP32 grouped launches (whose q-tiles with few live rows run trimmed)
    against the single builds of the same variant, bit for bit."""
    import paper_2012_15662_amd as rif
    ctx.set_tile_variant(variant)
    try:
        insts, items = make_items(rif.FP32)
        batch = ctx.batch(items, prec=rif.FP32)
        batch.run(use_graph=False)
        ctx.sync()
        for inst, (inp, npair, ncwo, _), out in zip(insts, items, batch.outs):
            print(f"case fp32 variant={variant} n_bf={inst.n_bf} pairs={npair}", flush=True)
            single = ctx.build_instance(inp, npair, ncwo, prec=rif.FP32)
            ctx.sync()
            for k in KEYS:
                assert np.array_equal(host(out[k]), host(single[k])), k
        batch.close()
    finally:
        ctx.set_tile_variant(-1)


@pytest.mark.parametrize("prec", [0, 3, 4])
def test_graph_replays(ctx, prec):
    import torch
    insts, items = make_items(prec)
    batch = ctx.batch(items, prec=prec)
    batch.run(use_graph=False)
    ctx.sync()
    eager = [{k: host(o[k]).copy() for k in KEYS} for o in batch.outs]
    for rep in range(4):
        for o in batch.outs:           # clobber the outputs between replays
            for k in KEYS:
                o[k].fill_(float("nan"))
        x = torch.randn(1024, 1024, device="cuda")
        y = (x @ x).sum()               # unrelated eager GPU work
        torch.cuda.synchronize()
        batch.run(use_graph=True)
        ctx.sync()
        for e, o in zip(eager, batch.outs):
            for k in KEYS:
                assert np.array_equal(e[k], host(o[k])), (rep, k)
        del y
    batch.close()


def test_batch_rejects_bad_instance(ctx):
    import paper_2012_15662_amd as rif
    insts, items = make_items(rif.FP64)
    inp, npair, ncwo, _ = items[0]
    bad = [(inp, npair, 200, None)]      # n_omega > n_mo
    with pytest.raises(ValueError):
        ctx.batch(bad)                   # binding refuses: tensors too small
    with pytest.raises(rif.RifError) as e:
        ctx.batch([(inp, 0, 1, None)])   # n_pairs = 0
    assert e.value.status == -1
