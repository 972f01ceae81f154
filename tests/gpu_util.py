"""Helpers for the GPU tests: upload synthetic instances, compare with the oracle."""
import numpy as np


def to_dev(inst, C=None):
    import torch
    dev = "cuda"
    return dict(
        b=torch.from_numpy(inst.b).to(dev),
        C=torch.from_numpy(inst.C if C is None else C).to(dev),
        H=torch.from_numpy(inst.H).to(dev),
        occ=torch.from_numpy(inst.occ).to(dev),
        pair_of=torch.from_numpy(inst.pair_of.astype(np.int32)).to(dev),
    )


def relerr(got, ref):
    """Normwise relative error max|got - ref| / max|ref|."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def host(t):
    return t.detach().cpu().numpy()
