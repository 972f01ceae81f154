"""The 64-molecule uneven batch that the batch bench times, against the oracle.

64 molecules, n_bf ~ U{60..400} (seed 3), n_aux = 3 n_bf, pairs = n_bf // 12,
Ncwo = 2, b drawn on the GPU per molecule (seeds 3000 + i).  The batch runs
as the bench runs it: autotuned tile shapes, one grouped launch per step,
replayed from a hipGraph.  Every molecule's energy, lambda, gradient, J and K
are compared with the FP64 oracle run on the same inputs copied to the host:

* FP64 to 1e-10 (relative energy, normwise arrays);
* split-BF16x6 within 1 uEh in energy and 1e-6 (normwise) in the gradient,
  the split-precision target, on every molecule;
* FP32 (plain FP32 MFMA, not a split mode) and split-FP16x3 do not meet
  1 uEh on every molecule (both are at FP32's level, about 1 uEh at these
  sizes): their errors are printed, with how many molecules meet the target,
  and only bounded (5 uEh, 1e-6) so that a regression fails.
"""
import numpy as np
import pytest

import synth
from oracle import pnof7_ri as ri
from tests.gpu_util import host, relerr

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
KEYS = ("J", "K", "lam", "grad")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    c = rif.Context()
    c.autotune(True)
    yield c
    c.close()


@pytest.fixture(scope="module")
def batch_and_refs():
    """Device inputs of the 64 molecules and the oracle's results for each."""
    items = synth.make_batch_device(64)
    refs = []
    for i, (inp, npair, ncwo) in enumerate(items):
        h = {k: host(v) for k, v in inp.items()}
        r = ri.build(h["b"], h["C"], h["H"], h["occ"], h["pair_of"], npair)
        refs.append({k: r[k] for k in KEYS + ("energy",)})
        if i % 16 == 15:
            print(f"oracle: {i + 1} of 64 molecules", flush=True)
    return items, refs


@pytest.mark.parametrize("prec_name", ["fp64", "bf16x6", "fp32", "fp16x3"])
def test_batch64_matches_oracle(ctx, batch_and_refs, prec_name):
    import paper_2012_15662_amd as rif
    prec = {"fp64": rif.FP64, "fp32": rif.FP32, "bf16x6": rif.BF16X6, "fp16x3": rif.FP16X3}[prec_name]
    bound_e = {"bf16x6": 1e-6, "fp32": 5e-6, "fp16x3": 5e-6}.get(prec_name)
    items, refs = batch_and_refs
    print(f"case batch64 prec={prec_name}", flush=True)
    batch = ctx.batch([(inp, npair, ncwo, None) for inp, npair, ncwo in items], prec=prec)
    batch.run(use_graph=True)
    batch.run(use_graph=True)        # a replay of the captured graph
    ctx.sync()
    worst = {"energy": 0.0, **{k: 0.0 for k in KEYS}}
    within = 0
    for i, (out, ref, (inp, npair, ncwo)) in enumerate(zip(batch.outs, refs, items)):
        e = float(host(out["energy"])[0])
        de = abs(e - ref["energy"])
        errs = {k: relerr(host(out[k]), ref[k]) for k in KEYS}
        if prec == rif.FP64:
            assert de <= 1e-10 * abs(ref["energy"]), (i, de)
            for k, v in errs.items():
                assert v <= 1e-10, (i, k, v)
        else:
            assert de <= bound_e, (i, inp["b"].shape[1], de)
            assert errs["grad"] <= 1e-6, (i, errs["grad"])
            within += de <= 1e-6
        worst["energy"] = max(worst["energy"], de)
        for k, v in errs.items():
            worst[k] = max(worst[k], v)
    print((f"{within} of 64 within 1 uEh; " if prec != rif.FP64 else "") + f"worst over 64: |dE| {worst['energy']:.2e} Eh, " +
          " ".join(f"{k} {v:.2e}" for k, v in worst.items() if k != "energy"), flush=True)
    batch.close()
