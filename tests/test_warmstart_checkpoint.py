"""The warm-start network's checkpoint format on the CPU: save() writes plain
arrays that load() reads back unchanged, and files of another layout are
refused.  No GPU work is involved in either; a stand-in context supplies the
parameter count (39*128 + 128 + 2*(128*128 + 128) + 128*7 + 7).
"""
import numpy as np
import pytest

from paper_2012_15662_amd import warmstart as ws

N_PARAMS = ws.N_IN * ws.N_HID + ws.N_HID + 2 * (ws.N_HID * ws.N_HID + ws.N_HID) + ws.N_HID * ws.N_OUT + ws.N_OUT


class _Ctx:
    def mlp_n_params(self):
        return N_PARAMS


def test_save_load_round_trip(tmp_path):
    import torch
    net = ws.WarmStartMLP(_Ctx(), seed=3, device="cpu")
    g = torch.Generator().manual_seed(5)
    net.m = torch.randn(N_PARAMS, generator=g)
    net.v = torch.rand(N_PARAMS, generator=g)
    net.step = 17
    mu = torch.randn(ws.N_IN, generator=g)
    sd = torch.rand(ws.N_IN, generator=g)
    path = tmp_path / "warm.npz"
    net.save(str(path), mu=mu, sigma=sd)
    back = ws.WarmStartMLP.load(_Ctx(), str(path), device="cpu")
    for k in ("theta", "m", "v"):
        assert torch.equal(getattr(back, k), getattr(net, k).float()), k
    assert back.step == 17
    assert torch.equal(back.mu, mu.float()) and torch.equal(back.sigma, sd.float())
    # without a standardisation the attributes come back as None
    net.save(str(path))
    back = ws.WarmStartMLP.load(_Ctx(), str(path), device="cpu")
    assert back.mu is None and back.sigma is None


def test_load_refuses_other_layouts(tmp_path):
    net = ws.WarmStartMLP(_Ctx(), seed=0, device="cpu")
    good = tmp_path / "good.npz"
    net.save(str(good))
    with np.load(str(good)) as f:
        arrs = {k: f[k] for k in f.files}
    cases = {
        "layers": dict(arrs, layers=np.array([39, 64, 64, 64, 7])),
        "theta": dict(arrs, theta=arrs["theta"][:-1]),
        "missing": {k: v for k, v in arrs.items() if k != "v"},
        "mu": dict(arrs, mu=np.zeros(5, np.float32)),
    }
    for name, a in cases.items():
        p = tmp_path / f"{name}.npz"
        np.savez(str(p), **a)
        with pytest.raises(ValueError):
            ws.WarmStartMLP.load(_Ctx(), str(p), device="cpu")
