"""Tile choices carried between contexts (rif_tune_report -> rif_tune_load).

A context that loads another context's report builds with the loaded variants
and times nothing again: its report after the build is the loaded text, and
its outputs equal the first context's bitwise.  A loaded variant that the
kernel does not have is ignored: that shape is timed as usual, and the build
is still correct.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import host, to_dev

pytestmark = pytest.mark.gpu
KEYS = ("energy", "lam", "grad", "Jn", "Kn")


def build(c, t, inst):
    out = c.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], inst.n_pairs, inst.n_cwo)
    c.sync()
    return {k: host(out[k]) for k in KEYS}


def test_loaded_choices_skip_timing():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    print("case tune load: 130/259/7/3", flush=True)
    inst = synth.make_instance(130, 259, 7, 3, 12)
    t = to_dev(inst)
    c1 = rif.Context()
    c1.autotune(True)
    ref = build(c1, t, inst)
    rep = c1.tune_report()
    assert rep.strip()
    c1.close()

    c2 = rif.Context()
    c2.autotune(True)
    c2.tune_load(rep)
    out = build(c2, t, inst)
    assert c2.tune_report() == rep          # no shape timed again
    for k in KEYS:
        assert np.array_equal(out[k], ref[k]), k
    c2.close()

    # a variant K^q does not have (it has two): that shape is timed afresh
    lines = rep.strip().splitlines()
    kao = [i for i, l in enumerate(lines) if l.startswith("kao ")]
    assert kao
    key = lines[kao[0]].split(" -> ")[0]
    lines[kao[0]] = key + " -> 3 | 1.0 1.0 1.0 1.0"
    c3 = rif.Context()
    c3.autotune(True)
    c3.tune_load("\n".join(lines) + "\n")
    out = build(c3, t, inst)
    after = c3.tune_report().strip().splitlines()
    assert sum(1 for l in after if l.startswith(key + " -> ")) == 2   # the loaded line and the timed one
    assert abs(out["energy"][0] - ref["energy"][0]) <= 1e-12 * abs(ref["energy"][0])
    assert np.max(np.abs(out["grad"] - ref["grad"])) <= 1e-12 * np.max(np.abs(ref["grad"]))
    with pytest.raises(rif.RifError):
        c3.tune_load("kao 1 2 -> x | 0.1")
    c3.close()
