"""rif_prepare_b (b from the three-centre integrals and the metric) against
the oracle (oracle/metric.py), through the C ABI.

The factorisation is compared where it is unique given the pivot rule: the
permutation exactly, L and D to 1e-10 (normwise), on SPD, indefinite,
2x2-forcing and singular metrics, up to 600 functions (several rows per
workgroup of the one-launch factorisation, with interchanges across and within
workgroups).  Up to about 1600 auxiliary functions it is the one-launch
factorisation; a 1640-function metric takes the per-column launches and is
checked the same way.  b is compared with the oracle's to a bound
scaled by kappa(G~) (the solve amplifies rounding by it), and the number of
raised eigenvalues exactly.  At full cyclohexane size (n_bf=348, n_aux=1044)
with an ill-conditioned, slightly indefinite metric: the same, plus the RI
identity checked on sampled (mu nu, sigma lambda) pairs.
"""
import numpy as np
import pytest

import synth
from oracle import metric as mt
from tests.gpu_util import host, relerr

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


def sym(n, seed, zero_diag=False):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n))
    A = (X + X.T) / 2
    if zero_diag:
        np.fill_diagonal(A, 0.0)
    return A


def run(ctx, T, G):
    import torch
    Td = torch.from_numpy(np.ascontiguousarray(T)).cuda()
    Gd = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    b, perm, L, D, nr = ctx.prepare_b(Td, Gd, factors=True)
    ctx.sync()
    return host(b), host(perm), host(L), host(D), int(host(nr)[0])


def b_tolerance(G, L, D, steps, delta):
    """Rounding bound for b = D~^(-1/2) L^-1 P^T T computed two ways: L^-1 amplifies
    by cond(L); an eigenvalue lambda of a D block carries the elimination's
    absolute error, about eps ||G||, so it is only as accurate as
    eps ||G|| / |lambda| (relative), which D~^(-1/2) carries into its rows."""
    g = np.max(np.abs(G))
    sens, k = 1.0, 0
    for s_ in steps:
        w = np.abs(np.linalg.eigvalsh(D[k:k + s_, k:k + s_]))
        sens = max(sens, g / max(w.min(), delta))
        k += s_
    return max(1e-12, 1e3 * 2.0 ** -52 * sens * np.linalg.cond(L))


def raised_count(D, steps, delta):
    k, n = 0, 0
    for s in steps:
        n += int(np.sum(np.linalg.eigvalsh(D[k:k + s, k:k + s]) < delta))
        k += s
    return n


@pytest.mark.parametrize("name,G", [
    ("spd", synth.make_metric(40, 1, cond=1e3)),
    ("indefinite", sym(37, 2)),
    ("forced_2x2", sym(30, 3, zero_diag=True)),
    ("indefinite_150", sym(150, 4)),
    ("forced_2x2_101", sym(101, 5, zero_diag=True)),
    ("one_aux", np.array([[2.5]])),
    ("indefinite_600", sym(600, 9)),
    ("forced_2x2_520", sym(520, 10, zero_diag=True)),
])
def test_factorisation_matches_oracle(ctx, name, G):
    print("case factorisation", name, G.shape, flush=True)
    n = G.shape[0]
    T = synth.make_three_centre(5, n, 10)
    b, perm, L, D, nr = run(ctx, T, G)
    p0, L0, D0, steps = mt.bunch_kaufman(G)
    assert np.array_equal(perm, p0)
    assert relerr(L, L0) < 1e-10 and relerr(D, D0) < 1e-10
    delta = mt.correction_threshold(G)
    assert nr == raised_count(D0, steps, delta)
    b0, _ = mt.prepare_b(T, G)
    err = relerr(b, b0)
    tol = b_tolerance(G, L0, D0, steps, delta)
    print("b rel err", err, "bound", tol, flush=True)
    assert err < tol
    assert np.array_equal(b, b.transpose(0, 2, 1))


def test_singular_column(ctx):
    G = sym(12, 6)
    G[:, 4] = 0.0
    G[4, :] = 0.0
    b, perm, L, D, nr = run(ctx, synth.make_three_centre(4, 12, 11), G)
    p0, L0, D0, _ = mt.bunch_kaufman(G)
    assert np.array_equal(perm, p0) and relerr(L, L0) < 1e-10 and relerr(D, D0) < 1e-10


def crafted_interchange(kind, n=300, seed=8):
    """A diagonally dominant metric whose first pivot step interchanges two rows
    held by one workgroup of the one-launch factorisation (256 workgroups, row
    i in workgroup i mod 256): a 1x1 pivot at row 256 (0 <-> 256), or a 2x2
    pivot on (0, 257) (1 <-> 257)."""
    rng = np.random.default_rng(seed)
    X = 0.01 * rng.standard_normal((n, n))
    G = (X + X.T) / 2 + np.diag(rng.uniform(1.0, 2.0, n))
    G[0, 0] = 1e-3
    if kind == "1x1":
        G[0, 256] = G[256, 0] = 1.0
        G[256, 256] = 5.0
    else:
        G[0, 257] = G[257, 0] = 1.0
        G[257, 257] = 1e-3
    return G


@pytest.mark.parametrize("kind", ["1x1", "2x2"])
def test_interchange_within_one_workgroup(ctx, kind):
    print("case factorisation interchange within a workgroup", kind, flush=True)
    G = crafted_interchange(kind)
    b, perm, L, D, nr = run(ctx, synth.make_three_centre(4, G.shape[0], 13), G)
    p0, L0, D0, steps = mt.bunch_kaufman(G)
    assert steps[0] == (1 if kind == "1x1" else 2)
    assert p0[0 if kind == "1x1" else 1] == (256 if kind == "1x1" else 257)
    assert np.array_equal(perm, p0)
    assert relerr(L, L0) < 1e-10 and relerr(D, D0) < 1e-10


def test_large_metric_takes_the_per_column_path(ctx):
    """1640 auxiliary functions: past what the one-launch factorisation holds in
    LDS, so the pivot and update launches per column run (indefinite metric,
    1x1 and 2x2 pivots)."""
    n = 1640
    print("case factorisation per-column path", n, flush=True)
    G = sym(n, 7)
    b, perm, L, D, nr = run(ctx, synth.make_three_centre(3, n, 12), G)
    p0, L0, D0, steps = mt.bunch_kaufman(G)
    assert 2 in steps and 1 in steps
    assert np.array_equal(perm, p0)
    assert relerr(L, L0) < 1e-10 and relerr(D, D0) < 1e-10


def test_full_size_ill_conditioned_metric(ctx):
    nb, na = 348, 1044
    print("case prepare_b full size n_bf=348 n_aux=1044", flush=True)
    G = synth.make_metric(na, 20, cond=1e10, n_negative=3)
    T = synth.make_three_centre(nb, na, 21)
    b, perm, L, D, nr = run(ctx, T, G)
    b0, info = mt.prepare_b(T, G)
    assert np.array_equal(perm, info["perm"])
    # L_ik = A_ik / d_k: a pivot d_k near eps ||G|| / tol leaves its column only
    # that accurate (the same sensitivity as b); D carries absolute rounding
    tol = b_tolerance(G, info["L"], info["D"], info["steps"], info["delta"])
    print("full-size L, D rel err", relerr(L, info["L"]), relerr(D, info["D"]), "bound", tol, flush=True)
    assert relerr(L, info["L"]) < tol and relerr(D, info["D"]) < 1e-12
    delta = info["delta"]
    assert nr == raised_count(info["D"], info["steps"], delta) and nr >= 3
    err = relerr(b, b0)
    tol = b_tolerance(G, info["L"], info["D"], info["steps"], delta)
    print("full-size b rel err", err, "bound", tol, "raised", nr, flush=True)
    assert err < tol
    # RI identity on sampled pairs: sum_k b^k_x b^k_y = T_x^T G~^-1 T_y
    Dt, _, _ = mt.corrected_blocks(info["D"], info["steps"], delta)
    Gt = mt.reconstruct(info["perm"], info["L"], Dt)
    rng = np.random.default_rng(22)
    Tm, bm = T.reshape(na, -1), b.reshape(na, -1)
    xs = rng.choice(nb * nb, 40, replace=False)
    lhs = bm[:, xs].T @ bm[:, xs]
    rhs = Tm[:, xs].T @ np.linalg.solve(Gt, Tm[:, xs])
    assert np.max(np.abs(lhs - rhs)) <= 1e-5 * np.max(np.abs(rhs))
    # Backward error of the solve with the GPU's own factors: b^T = D~^-1/2 L^-1 P^T T
    # with L^-1 formed by forward substitution, then one GEMM, so the residual of
    # P L D~^1/2 b^T = T obeys |T_pi - L D~^1/2 b^T| <= c n eps |L| |L^-1| |T_pi|
    # elementwise, however small the pivots (sampled columns, c = 4)
    _, Dh, _ = mt.corrected_blocks(D, info["steps"], delta)
    cols = rng.choice(nb * nb, 400, replace=False)
    Tp = Tm[perm][:, cols]
    R = Tp - L @ (Dh @ bm[:, cols])
    bound = 4.0 * na * np.finfo(float).eps * (np.abs(L) @ (np.abs(np.linalg.inv(L)) @ np.abs(Tp)))
    ratio = np.max(np.abs(R) / bound)
    print("full-size backward error: max |R| / (4 n eps |L||L^-1||T|) =", ratio,
          " normwise |R|/(|L||D^1/2 b^T|) =", np.max(np.abs(R)) / np.max(np.abs(L) @ np.abs(Dh @ bm[:, cols])),
          flush=True)
    assert ratio <= 1.0


def test_prepared_b_feeds_the_build(ctx):
    """End to end: T, G -> b (rif_prepare_b) -> rif_build, against the oracle's
    b and build (well-conditioned metric, so b is accurate to rounding)."""
    import torch
    from oracle import pnof7_ri as ri
    nb, na, npair, ncwo = 40, 120, 3, 2
    G = synth.make_metric(na, 30, cond=1e4)
    T = synth.make_three_centre(nb, na, 31)
    inst = synth.make_instance(nb, na, npair, ncwo, 32)
    bd = ctx.prepare_b(torch.from_numpy(T).cuda(), torch.from_numpy(G).cuda())
    C, H = torch.from_numpy(inst.C).cuda(), torch.from_numpy(inst.H).cuda()
    occ, pm = torch.from_numpy(inst.occ).cuda(), torch.from_numpy(inst.pair_of.astype(np.int32)).cuda()
    out = ctx.build(bd, C, H, occ, pm, npair, ncwo)
    ctx.sync()
    b0, _ = mt.prepare_b(T, G)
    ref = ri.build(b0, inst.C, inst.H, inst.occ, inst.pair_of, npair)
    assert relerr(host(bd), b0) < 1e-12
    assert abs(float(host(out["energy"])[0]) - ref["energy"]) <= 1e-10 * abs(ref["energy"])
    assert relerr(host(out["grad"]), ref["grad"]) < 1e-10
