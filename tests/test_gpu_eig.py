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
zero matrix, degenerate eigenvalues and the sizes at its limits.  The
library's divide and conquer (kind 3) runs on the same matrices and on
tridiagonal ones (which the reduction passes through unchanged) chosen for
its merge paths: Toeplitz and glued Wilkinson matrices (many rotation
deflations), decoupled and weakly coupled clusters (deflation by small update
components), a zero coupling at a split point, sizes around the leaf size
of 16 rows and the merge tree's uneven splits, and a non-finite F, which it
reports as info = 1 without disturbing the next call.
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
@pytest.mark.parametrize("kind", [1, 2, 3])
def test_random_matrices(ctx, n, kind):
    print("case eig random", n, "kind", kind, flush=True)
    F = random_sym(n, 100 + n)
    w, V = diagonalise(ctx, F, kind)
    check(F, w, V)


@pytest.mark.parametrize("groups", [18, 23, 64, 255])
@pytest.mark.parametrize("kind", [2, 3])
def test_workgroup_counts_agree(ctx, groups, kind):
    print("case eig groups", groups, "kind", kind, flush=True)
    F = random_sym(348, 7)
    w, V = diagonalise(ctx, F, kind, groups)
    check(F, w, V)
    w1, V1 = diagonalise(ctx, F, 1)
    assert np.max(np.abs(w - w1)) <= 8 * 348 * EPS * np.max(np.abs(w1))


@pytest.mark.parametrize("kind", [2, 3])
def test_diagonal_and_reducible(ctx, kind):
    print("case eig diagonal / reducible, kind", kind, flush=True)
    rng = np.random.default_rng(3)
    d = rng.permutation(np.linspace(-4.0, 5.0, 90))
    F = np.diag(d)
    w, V = diagonalise(ctx, F, kind)
    check(F, w, V)
    assert np.array_equal(np.abs(V), np.eye(90)[:, np.argsort(d)])   # every reflector the identity
    # two uncoupled blocks, the second starting with a zero column below the diagonal
    F = np.zeros((70, 70))
    F[:40, :40] = random_sym(40, 4)
    F[40:, 40:] = random_sym(30, 5, spread=3.0) + 20.0 * np.eye(30)
    w, V = diagonalise(ctx, F, kind)
    check(F, w, V)


@pytest.mark.parametrize("kind", [2, 3])
def test_zero_and_degenerate(ctx, kind):
    print("case eig zero / degenerate, kind", kind, flush=True)
    F = np.zeros((33, 33))
    w, V = diagonalise(ctx, F, kind)
    assert np.all(w == 0.0)
    check(F, w, V, distinct=False)
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.standard_normal((120, 120)))
    lam = np.repeat([-2.0, 0.5, 3.0], 40)
    F = (Q * lam) @ Q.T
    F = 0.5 * (F + F.T)
    w, V = diagonalise(ctx, F, kind)
    check(F, w, V, distinct=False)


def tridiag(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def glued_wilkinson(m, copies, glue):
    # copies of W_m^+ (|i - m/2| on the diagonal, ones beside it) joined by `glue`:
    # pairs of eigenvalues agreeing to many digits
    d = np.tile(np.abs(np.arange(m) - (m - 1) / 2.0), copies)
    e = np.ones(m * copies - 1)
    e[m - 1::m] = glue
    return tridiag(d, e)


@pytest.mark.parametrize("case", ["toeplitz", "wilkinson", "glued", "clusters", "split_zero", "graded"])
def test_divide_and_conquer_paths(ctx, case):
    print("case eig dc", case, flush=True)
    rng = np.random.default_rng(21)
    distinct = True
    if case == "toeplitz":      # 2 on the diagonal, 1 beside it: closed-form spectrum
        n = 200
        F = tridiag(np.full(n, 2.0), np.ones(n - 1))
        w_exact = 2.0 + 2.0 * np.cos(np.pi * np.arange(n, 0, -1) / (n + 1))
    elif case == "wilkinson":
        F = tridiag(np.abs(np.arange(101) - 50.0), np.ones(100))
        distinct = False        # its top pairs agree to more digits than the gap test resolves
    elif case == "glued":
        F = glued_wilkinson(21, 16, 1e-7)
        distinct = False
    elif case == "clusters":    # six clusters of 58, coupled at 1e-8
        d = np.repeat(rng.standard_normal(6), 58) + 1e-3 * rng.standard_normal(348)
        F = tridiag(d, 1e-8 * rng.standard_normal(347))
        distinct = False
    elif case == "split_zero":  # zero coupling at the top split point and at leaf boundaries
        e = rng.standard_normal(347)
        e[173] = 0.0
        e[21::22] = 0.0
        F = tridiag(rng.standard_normal(348), e)
    else:                       # entries graded over 12 orders of magnitude
        n = 130
        F = tridiag(np.logspace(0, -12, n) * rng.choice([-1.0, 1.0], n), np.logspace(0, -12, n - 1))
    w, V = diagonalise(ctx, F, 3)
    check(F, w, V, distinct=distinct)
    if case == "toeplitz":
        assert np.max(np.abs(w - w_exact)) <= 64 * EPS * 4.0
    w2, _ = diagonalise(ctx, F, 2)
    assert np.max(np.abs(w - w2)) <= 8 * F.shape[0] * EPS * np.max(np.abs(w2))


@pytest.mark.parametrize("n", [32, 33, 63, 64, 65, 129, 255, 257, 580])
def test_divide_and_conquer_sizes(ctx, n):
    print("case eig dc size", n, flush=True)
    F = random_sym(n, 300 + n)
    w, V = diagonalise(ctx, F, 3)
    check(F, w, V)


def test_size_limits(ctx):
    import paper_2012_15662_amd as rif
    print("case eig size limits", flush=True)
    F = np.array([[2.5]])
    w, V = diagonalise(ctx, F, 0)          # n = 1: the automatic choice takes dsyevd
    assert w[0] == 2.5 and abs(V[0, 0]) == 1.0
    for kind in (2, 3):
        with pytest.raises(rif.RifError):
            diagonalise(ctx, F, kind)
    with pytest.raises(rif.RifError):
        ctx.set_eigensolver(4)
    F = random_sym(1500, 11)               # rows do not fit: TRD and DC refuse, AUTO falls back
    for kind in (2, 3):
        with pytest.raises(rif.RifError):
            diagonalise(ctx, F, kind)
    w, V = diagonalise(ctx, F, 0)
    check(F, w, V)
    F = random_sym(1000, 12)               # near the largest that fits (256 workgroups)
    for kind in (2, 3):
        w, V = diagonalise(ctx, F, kind)
        check(F, w, V)


@pytest.mark.parametrize("where", ["off-diagonal NaN", "diagonal inf"])
def test_divide_and_conquer_reports_non_finite_input(ctx, where):
    import torch
    print("case eig dc non-finite:", where, flush=True)
    n = 40
    F = random_sym(n, 5)
    lam = np.tril(F, -1)
    eps = np.ascontiguousarray(np.diag(F)).copy()
    if where == "off-diagonal NaN":
        lam[7, 3] = np.nan
    else:
        eps[11] = np.inf
    C = torch.eye(n, dtype=torch.float64, device="cuda")
    info = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    ctx.set_eigensolver(3)
    ctx.orbital_step(torch.from_numpy(lam).cuda(), C, n, eps_in=torch.from_numpy(eps).cuda(), info=info)
    ctx.sync()
    assert int(host(info)[0]) == 1
    w, V = diagonalise(ctx, F, 3)   # the next call is unaffected
    check(F, w, V)
