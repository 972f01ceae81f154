"""The orbital step's eigensolvers (rif_set_eigensolver) on chosen symmetric
matrices.

rif_orbital_step diagonalises F with F_pq = lambda_{hi,lo} - lambda_{lo,hi}
off the diagonal and eps_in on it.  With n_omega = n_mo and lambda holding the
wanted F below its diagonal (zero above), F is any symmetric matrix; with C = I
(n_bf = n_mo) C comes back as the eigenvectors V.  Checked against LAPACK's
eigh (numpy): eigenvalues to a few ulps of ||F||, eigenvectors up to sign to
the perturbation bound eps ||F|| / gap where the eigenvalues are separated, and
for every case orthonormality of V and the residual F V - V diag(w).  The
tridiagonal reduction (one cooperative launch) is checked at several workgroup
counts, on a diagonal matrix (every reflector the identity), a reducible one, a
zero matrix, degenerate eigenvalues and the sizes at its limits.
"""
import numpy as np
import pytest

from tests.gpu_util import host

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2012_15662_amd as rif
    c = rif.Context()
    yield c
    c.set_eigensolver(rif.EIG_AUTO)
    c.close()


def diagonalise(ctx, F, kind, groups=0):
    import torch
    n = F.shape[0]
    lam = np.tril(F, -1)
    C = torch.eye(n, dtype=torch.float64, device="cuda")
    info = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    ctx.set_eigensolver(kind, groups)
    w = ctx.orbital_step(torch.from_numpy(lam).cuda(), C, n,
                         eps_in=torch.from_numpy(np.ascontiguousarray(np.diag(F))).cuda(), info=info)
    ctx.sync()
    assert int(host(info)[0]) == 0
    return host(w), host(C)


def check(F, w, V, distinct=True):
    n = F.shape[0]
    wr, Vr = np.linalg.eigh(F)
    nrm = max(np.linalg.norm(F, 2), 1e-300)
    assert np.all(np.diff(w) >= 0), "eigenvalues ascending"
    assert np.max(np.abs(w - wr)) <= 8 * n * EPS * nrm + 1e-300
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 16 * n * EPS
    assert np.max(np.abs(F @ V - V * w)) <= 16 * n * EPS * nrm + 1e-300
    if distinct:
        gap = np.min(np.diff(wr))
        s = np.sign(np.sum(V * Vr, axis=0))
        s[s == 0] = 1
        assert np.max(np.abs(V * s - Vr)) <= 64 * n * EPS * nrm / gap


def random_sym(n, seed, spread=10.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w = np.sort(rng.uniform(-spread, spread, n))
    return (Q * w) @ Q.T


@pytest.mark.parametrize("n", [2, 3, 17, 100, 348, 501])
@pytest.mark.parametrize("kind", [1, 2])
def test_random_matrices(ctx, n, kind):
    print("case eig random", n, "kind", kind, flush=True)
    F = random_sym(n, 100 + n)
    w, V = diagonalise(ctx, F, kind)
    check(F, w, V)


@pytest.mark.parametrize("groups", [18, 23, 64, 255])
def test_workgroup_counts_agree(ctx, groups):
    print("case eig groups", groups, flush=True)
    F = random_sym(348, 7)
    w, V = diagonalise(ctx, F, 2, groups)
    check(F, w, V)
    w1, V1 = diagonalise(ctx, F, 1)
    assert np.max(np.abs(w - w1)) <= 8 * 348 * EPS * np.max(np.abs(w1))


def test_diagonal_and_reducible(ctx):
    print("case eig diagonal / reducible", flush=True)
    rng = np.random.default_rng(3)
    d = rng.permutation(np.linspace(-4.0, 5.0, 90))
    F = np.diag(d)
    w, V = diagonalise(ctx, F, 2)
    check(F, w, V)
    assert np.array_equal(np.abs(V), np.eye(90)[:, np.argsort(d)])   # every reflector the identity
    # two uncoupled blocks, the second starting with a zero column below the diagonal
    F = np.zeros((70, 70))
    F[:40, :40] = random_sym(40, 4)
    F[40:, 40:] = random_sym(30, 5, spread=3.0) + 20.0 * np.eye(30)
    w, V = diagonalise(ctx, F, 2)
    check(F, w, V)


def test_zero_and_degenerate(ctx):
    print("case eig zero / degenerate", flush=True)
    F = np.zeros((33, 33))
    w, V = diagonalise(ctx, F, 2)
    assert np.all(w == 0.0)
    check(F, w, V, distinct=False)
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.standard_normal((120, 120)))
    lam = np.repeat([-2.0, 0.5, 3.0], 40)
    F = (Q * lam) @ Q.T
    F = 0.5 * (F + F.T)
    w, V = diagonalise(ctx, F, 2)
    check(F, w, V, distinct=False)


def test_size_limits(ctx):
    import paper_2012_15662_amd as rif
    print("case eig size limits", flush=True)
    F = np.array([[2.5]])
    w, V = diagonalise(ctx, F, 0)          # n = 1: the automatic choice takes dsyevd
    assert w[0] == 2.5 and abs(V[0, 0]) == 1.0
    with pytest.raises(rif.RifError):
        diagonalise(ctx, F, 2)
    with pytest.raises(rif.RifError):
        ctx.set_eigensolver(3)
    F = random_sym(1500, 11)               # rows do not fit: TRD refuses, AUTO falls back
    with pytest.raises(rif.RifError):
        diagonalise(ctx, F, 2)
    w, V = diagonalise(ctx, F, 0)
    check(F, w, V)
    F = random_sym(1000, 12)               # near the largest that fits (256 workgroups)
    w, V = diagonalise(ctx, F, 2)
    check(F, w, V)
