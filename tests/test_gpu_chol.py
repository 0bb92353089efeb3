"""GPU blocked Cholesky factorisation (the left Gram factor of the simultaneous
truncation) against LAPACK and by reconstruction, for one and several panels of 32
columns, full-rank, rank-deficient, graded and nearly-identity Gram matrices."""
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


def _gram(n, r, rng, scale=None):
    b = rng.standard_normal((n, r))
    if scale is not None:
        b *= scale[None, :]
    return b @ b.T


@pytest.mark.parametrize("n", [1, 5, 31, 32, 33, 64, 100, 257, 540])
def test_cholesky_full_rank_matches_lapack(ctx, n):
    rng = np.random.default_rng(n)
    A = _gram(n, n, rng) + 0.1 * np.eye(n)
    W = ctx.cholesky(A)
    ref = np.linalg.cholesky(A)
    an = np.abs(A).max()
    assert np.all(np.triu(W, 1) == 0.0)
    assert np.abs(W @ W.T - A).max() <= 1e-12 * an * max(1, n / 100)
    assert np.abs(W - ref).max() <= 1e-9 * np.sqrt(an)


@pytest.mark.parametrize("n,r", [(40, 7), (100, 60), (300, 150), (540, 270)])
def test_cholesky_rank_deficient_drops_dependent_columns(ctx, n, r):
    rng = np.random.default_rng(1000 + n)
    A = _gram(n, r, rng)
    W = ctx.cholesky(A)
    an = np.abs(A).max()
    assert np.all(np.triu(W, 1) == 0.0)
    assert np.abs(W @ W.T - A).max() <= 1e-10 * an
    # the first r columns of a generic Gram of rank r are independent, the rest depend on them
    nz = int(np.sum(np.abs(W).max(axis=0) > 0))
    assert nz == r


@pytest.mark.parametrize("n", [64, 200, 450])
def test_cholesky_graded_and_near_identity(ctx, n):
    rng = np.random.default_rng(7 * n)
    A = _gram(n, n, rng, scale=np.logspace(0, -5, n))
    W = ctx.cholesky(A)
    assert np.abs(W @ W.T - A).max() <= 1e-10 * np.abs(A).max()
    B = np.eye(n) + 1e-12 * (lambda m: (m + m.T) / 2)(rng.standard_normal((n, n)))
    W = ctx.cholesky(B)
    assert np.abs(W @ W.T - B).max() <= 1e-14
    assert np.abs(W - np.eye(n)).max() <= 1e-11
