"""GPU eigensolvers behind the Gram factorisations (Jacobi and tridiagonal), checked
against LAPACK (numpy.linalg.eigh) and by residual/orthogonality on structured input:
dense random, rank deficient Grams, graded spectra, exact degeneracy, clusters and
block-diagonal matrices."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

native = pytest.importorskip("paper_2604_16118_amd.native")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = native.Context(0)
    yield c
    c.close()


def _rand_sym(n, rng):
    a = rng.standard_normal((n, n))
    return (a + a.T) / 2


def _gram(n, r, rng, graded=False):
    b = rng.standard_normal((n, r))
    if graded:
        b *= np.logspace(0, -7, r)[None, :]
    return b @ b.T


def _spectrum(w_ref, n, rng, clusters=False):
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (q * w_ref) @ q.T


def _block_diag(n, rng):
    a = np.zeros((n, n))
    i = 0
    while i < n:
        k = min(n - i, int(rng.integers(1, 9)))
        a[i:i + k, i:i + k] = _gram(k, max(1, k - 2), rng)
        i += k
    p = rng.permutation(n)
    return a[np.ix_(p, p)]


def _zero_rows(n, rng):
    a = _gram(n, max(1, n // 2), rng, graded=True)
    z = rng.random(n) < 0.3
    a[z, :] = 0.0
    a[:, z] = 0.0
    return a


CASES = {
    "rand": lambda n, rng: _rand_sym(n, rng),
    "gram_rankdef": lambda n, rng: _gram(n, max(1, n // 5), rng),
    "gram_graded": lambda n, rng: _gram(n, max(1, n // 2), rng, graded=True),
    "degenerate": lambda n, rng: _spectrum(np.repeat(np.arange(1, 1 + (n + 2) // 3), 3)[:n].astype(float), n, rng),
    "cluster": lambda n, rng: _spectrum(np.concatenate([1 + 1e-11 * np.arange(n // 2), np.linspace(2, 3, n - n // 2)]), n, rng),
    "blockdiag": _block_diag,
    # Gram matrices of nearly orthonormal vectors: identity plus 1e-12 noise, and a
    # narrow band about 5 (spread 1e-6)
    "near_identity": lambda n, rng: np.eye(n) + 1e-12 * _rand_sym(n, rng),
    # congruence W^T G W with a triangular factor W that has zero columns: exact zero rows
    # and columns scattered through the matrix
    "zero_rows": lambda n, rng: _zero_rows(n, rng),
    "narrow_band": lambda n, rng: 5 * np.eye(n) + 1e-6 * _rand_sym(n, rng),
    # n/2 pairs 1e-12 apart: the largest possible number of eigenvector clusters (each pair
    # is solved and orthogonalised cooperatively)
    "pairs": lambda n, rng: _spectrum(np.repeat(np.linspace(1, 2, (n + 1) // 2), 2)[:n]
                                      + 1e-12 * np.tile([0.0, 1.0], (n + 1) // 2)[:n], n, rng),
}


def _cluster_width(wr, tol):
    """Largest spread of a chain of eigenvalues whose neighbours are within tol."""
    wr = np.sort(wr)
    best, start = 0.0, 0
    for i in range(1, len(wr) + 1):
        if i == len(wr) or wr[i] - wr[i - 1] > tol:
            best = max(best, wr[i - 1] - wr[start])
            start = i
    return best


def _check(A, w, V, method):
    """Jacobi (method 0): eigenpairs to working accuracy, V orthogonal to 1e-10.
    Tridiagonal (method 1): inverse iteration resolves a gap g_j = min(1e-7 ||A||,
    0.01 |lambda_j|) to each neighbour, so |v_i^T v_j| is about eps ||A|| / min(g_i, g_j)
    (tolerance 100 eps ||A|| / min(g_i, g_j)); vectors of closer eigenvalues are
    orthogonalised against each other and span their chain's invariant subspace, so the
    residual is bounded by the chain's width; V Lambda V^T reproduces A to 1e-10 ||A||;
    eigenvalues at or below 1e-12 max |lambda| carry zero vectors."""
    n = A.shape[0]
    wr = np.linalg.eigvalsh(A)[::-1]
    an = max(np.abs(wr).max(), 1e-300)
    sz = max(1.0, n / 100)
    assert np.all(np.diff(w) <= 1e-12 * an), "eigenvalues not descending"
    assert np.abs(w - wr).max() <= 1e-12 * an * sz
    if method == 0:
        keep = np.arange(n)
        res_tol = 1e-11 * an * sz
        orth_tol = np.full((n, n), 1e-10 * sz)
    else:
        keep = np.nonzero(np.abs(w) > 1e-12 * an)[0]
        for j in np.setdiff1d(np.arange(n), keep):
            assert np.linalg.norm(V[:, j]) == 0.0
        res_tol = 1e-11 * an * sz + _cluster_width(wr, 1e-7 * an)
        g = np.minimum(1e-7 * an, 1e-2 * np.abs(w[keep]))
        orth_tol = 100 * 2.2e-16 * an / np.minimum.outer(g, g) + 1e-10 * sz
        recon = (V[:, keep] * w[keep]) @ V[:, keep].T
        assert np.abs(recon - A).max() <= 1e-10 * an * sz
    Vk = V[:, keep]
    res = A @ Vk - Vk * w[keep]
    assert np.abs(res).max() <= res_tol
    assert np.all(np.abs(Vk.T @ Vk - np.eye(len(keep))) <= orth_tol)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("kind", sorted(CASES))
@pytest.mark.parametrize("n", [1, 2, 7, 41, 64, 130, 257])
def test_sym_eig(ctx, method, kind, n):
    rng = np.random.default_rng(1000 * n + sorted(CASES).index(kind))
    A = CASES[kind](n, rng)
    A = (A + A.T) / 2
    w, V = ctx.sym_eig(A, method)
    _check(A, w, V, method)


@pytest.mark.parametrize("kind", sorted(CASES))
@pytest.mark.parametrize("n", [538, 1024])
def test_sym_eig_at_gram_sizes_of_the_workload(ctx, kind, n):
    """The tridiagonal solver at the sizes the L = 48, cap 512 Grams reach (about 538) and
    at its limit of 1024."""
    rng = np.random.default_rng(1000 * n + sorted(CASES).index(kind))
    A = CASES[kind](n, rng)
    A = (A + A.T) / 2
    w, V = ctx.sym_eig(A, 1)
    _check(A, w, V, 1)


@pytest.mark.parametrize("kind", ["rand", "gram_graded", "cluster", "degenerate", "zero_rows"])
@pytest.mark.parametrize("n", [2, 3, 41, 130, 192, 193, 257, 538])
def test_sym_eig_step_and_panel_reductions_agree(ctx, kind, n):
    """The two reductions to tridiagonal form (one Householder step per launch on several
    workgroups, and panels of 32 steps on one workgroup with GEMM trailing updates) each
    pass the checks, and their eigenvalues agree to rounding."""
    rng = np.random.default_rng(9000 + n + sorted(CASES).index(kind))
    A = CASES[kind](n, rng)
    A = (A + A.T) / 2
    out = {}
    try:
        for name, limit in (("steps", 1 << 30), ("panels", 0)):
            ctx.set_tridiag_steps(limit)
            out[name] = ctx.sym_eig(A, 1)
            _check(A, *out[name], 1)
    finally:
        ctx.set_tridiag_steps(native.TRIDIAG_STEPS_DEFAULT)
    an = max(np.abs(np.linalg.eigvalsh(A)).max(), 1e-300)
    assert np.abs(out["steps"][0] - out["panels"][0]).max() <= 1e-13 * an * max(1.0, n / 100)


@pytest.mark.parametrize("method", [0, 1])
def test_sym_eig_zero_and_diagonal(ctx, method):
    n = 50
    w, V = ctx.sym_eig(np.zeros((n, n)), method)
    assert np.all(w == 0.0)
    d = np.linspace(-3, 5, n)
    w, V = ctx.sym_eig(np.diag(d), method)
    assert np.abs(w - d[::-1]).max() <= 1e-14 * 5
    nz = np.abs(w) > 1e-12 * 5
    assert np.abs(np.abs(V[:, nz]).max(axis=0) - 1).max() <= 1e-12


@pytest.mark.parametrize("kind", ["rand", "gram_graded", "cluster", "degenerate", "zero_rows"])
@pytest.mark.parametrize("n,nvec", [(41, 0), (41, 7), (130, 65), (257, 1), (257, 256), (300, 300), (538, 270),
                                    (1024, 512), (1024, 1024)])
def test_sym_eig_top(ctx, kind, n, nvec):
    """Leading eigenvectors only: the eigenvalues are those of the full solve, the first
    nvec columns pass the same checks, the rest are zero."""
    rng = np.random.default_rng(7000 + n + 13 * nvec + sorted(CASES).index(kind))
    A = CASES[kind](n, rng)
    A = (A + A.T) / 2
    w_all, V_all = ctx.sym_eig(A, 1)
    w, V = ctx.sym_eig(A, 1, nvec=nvec)
    assert np.array_equal(w, w_all)
    assert np.all(V[:, nvec:] == 0.0)
    # the computed columns come from the same inverse iteration, except inside clusters
    # cut by nvec, where they are orthogonalised against fewer members
    wr = np.linalg.eigvalsh(A)[::-1]
    an = max(np.abs(wr).max(), 1e-300)
    keep = [j for j in range(nvec) if abs(w[j]) > 1e-12 * an]
    Vk = V[:, keep]
    res = A @ Vk - Vk * w[keep]
    assert np.abs(res).max(initial=0.0) <= 1e-11 * an * max(1.0, n / 100) + _cluster_width(wr, 1e-7 * an)
    g = np.minimum(1e-7 * an, 1e-2 * np.abs(w[keep]))
    orth_tol = 100 * 2.2e-16 * an / np.minimum.outer(g, g) + 1e-10 * max(1.0, n / 100)
    assert np.all(np.abs(Vk.T @ Vk - np.eye(len(keep))) <= orth_tol)


def test_sym_eig_top_rejects_bad_count(ctx):
    with pytest.raises(Exception):
        ctx.sym_eig(np.eye(4), 1, nvec=5)
