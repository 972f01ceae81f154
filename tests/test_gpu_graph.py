"""One rif_build captured in a hipGraph (torch.cuda.graph on the context's
stream; the build forks its side stream with events, which the capture
follows) and replayed: every replay, with unrelated eager GPU work and
synchronisations between replays and the outputs overwritten by NaN, must
reproduce the eager build bit for bit.  The build allocates nothing and sets
no memory once its workspace exists, so the graph holds kernel nodes only.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import host, to_dev

pytestmark = pytest.mark.gpu
KEYS = ("b_half", "b_mo", "d", "J", "K", "Jn", "Kn", "energy", "lam", "grad")


@pytest.mark.parametrize("prec", [0, 3])
def test_captured_build_replays_bitwise(prec):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    print(f"case graph capture prec={prec} 130/259/7/3", flush=True)
    inst = synth.make_instance(130, 259, 7, 3, 21)
    t = to_dev(inst)
    s = torch.cuda.Stream()
    ctx = rif.Context(stream=s)
    try:
        with torch.cuda.stream(s):
            out = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec)
        torch.cuda.synchronize()
        eager = {k: host(out[k]).copy() for k in KEYS}
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo, prec=prec, out=out)
        torch.cuda.synchronize()
        for rep in range(3):
            for k in KEYS:
                out[k].fill_(float("nan"))
            x = torch.randn(512, 512, device="cuda")
            y = (x @ x).sum()            # unrelated eager GPU work
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for k in KEYS:
                assert np.array_equal(host(out[k]), eager[k]), (rep, k)
            del y
        del g
    finally:
        ctx.close()
