"""Host-side arithmetic of bench.py (CPU): the flop counts behind the reported
TFLOP/s and rooflines.

A build's algorithmic flops are the sum over its distinct steps, symmetric
outputs counted once: half transform 2 A B^2 W, MO transform 2 A B W^2,
J/K-MO 4 A W^2, J^q and K^q A W B (B + 1) each, Fock 4 W^2 B^2, H C_Omega
2 B^2 W and lambda 2 N_mo B W (A = n_aux, B = n_bf, W = n_omega).  The
pre-split kernels repeat the same arithmetic, so their table entries must
equal their split-on-load counterparts and must not be added to a build.
"""
import bench


def test_build_flops_counts_each_step_once():
    for nb, na, nw, nmo in ((348, 1044, 120, 348), (580, 1740, 200, 580), (1000, 3000, 420, 1000), (17, 5, 3, 9)):
        kf = bench.kernel_flops(nb, na, nw, nmo)
        assert kf["half_transform_presplit"] == kf["half_transform"]
        assert kf["jao_presplit"] == kf["jao"]
        steps = (2 * na * nb * nb * nw + 2 * na * nb * nw * nw + 4 * na * nw * nw
                 + 2 * na * nw * nb * (nb + 1) + 4 * nw * nw * nb * nb + 2 * nb * nb * nw + 2 * nmo * nb * nw)
        assert bench.build_flops(nb, na, nw, nmo) == float(steps)


def test_cyclohexane_build_count():
    # the figure the design notes quote for the cyclohexane-like build
    assert round(bench.build_flops(348, 1044, 120, 348) / 1e10, 2) == 7.83
