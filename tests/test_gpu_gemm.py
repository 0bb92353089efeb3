"""Grouped block GEMM (the operator contractions) through pv_gemm, against NumPy: tile
grids from one to thousands of tiles (with the XCD-grouped tile order and its ragged
end), the split-K path for tall K, both operand orientations, ragged edges, alpha/beta,
and the float32 variant."""
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


# (M, N, K): small, both long, short M with long N, short N with long M, tall K (split-K),
# tiny and ragged
SHAPES = [(100, 90, 37), (1100, 1030, 70), (200, 2000, 45), (2000, 200, 45), (100, 1500, 33),
          (120, 96, 5000), (1, 1, 1), (65, 129, 17), (300, 5000, 19), (5000, 300, 19)]


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K", SHAPES)
def test_gemm_float64(ctx, M, N, K, ta, tb):
    rng = np.random.default_rng(M * 7 + N * 3 + K + 11 * ta + 5 * tb)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    ref = -0.5 * (A.T if ta else A) @ (B.T if tb else B) + 2.0 * C0
    out = ctx.gemm(A, B, C0, ta=ta, tb=tb, alpha=-0.5, beta=2.0)
    # float64 accumulation: error ~ K eps |A||B|
    tol = 1e-14 * K * np.abs(A).max() * np.abs(B).max() + 1e-15 * np.abs(ref).max()
    assert np.abs(out - ref).max() <= tol


@pytest.mark.parametrize("M,N,K", [(100, 90, 37), (200, 2000, 45), (2000, 200, 45), (1100, 1030, 70)])
def test_gemm_float32(ctx, M, N, K):
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    ref = A @ B
    out = ctx.gemm(A, B, precision=1)
    # operands rounded to float32 (relative 6e-8 each), float32 accumulation over K terms
    tol = 4e-7 * np.sqrt(K) * np.abs(A).max() * np.abs(B).max() * 4
    assert np.abs(out - ref).max() <= tol
    assert np.abs(out - ref).max() > 0  # it did run in float32


def _bf16(x):
    """Round to the nearest bfloat16 (ties to even) through float32, as the kernel does."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(100, 90, 37), (200, 2000, 45), (2000, 200, 45), (1100, 1030, 70),
                                   (65, 129, 17), (120, 96, 5000)])
def test_gemm_bfloat16(ctx, M, N, K, ta, tb):
    """Operands rounded to bfloat16 and float32 accumulation: against the exact product of
    the rounded operands, the error is the float32 accumulation alone; against the
    float64 product it is the operand rounding (8 bits)."""
    rng = np.random.default_rng(M + 3 * N + 7 * K + ta)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    Ab, Bb = _bf16(A), _bf16(B)
    ref_b = 1.5 * (Ab.T if ta else Ab) @ (Bb.T if tb else Bb) - 0.5 * C0
    out = ctx.gemm(A, B, C0, ta=ta, tb=tb, alpha=1.5, beta=-0.5, precision=2)
    amax, bmax = np.abs(A).max(), np.abs(B).max()
    assert np.abs(out - ref_b).max() <= 1.5 * 4 * 6e-8 * np.sqrt(K) * amax * bmax * 4
    ref = 1.5 * (A.T if ta else A) @ (B.T if tb else B) - 0.5 * C0
    err = np.abs(out - ref).max()
    assert 0 < err <= 1.5 * 2 * 4e-3 * np.sqrt(K) * amax * bmax * 4
    t = ctx.timers()
    assert t["gemm_bf16_mfma"]["calls"] > 0


def test_gemm_rejects_bad_arguments(ctx):
    with pytest.raises(Exception):
        ctx.gemm(np.ones((3, 2)), np.ones((3, 2)))  # inner dimensions differ
    with pytest.raises(Exception):
        ctx.gemm(np.ones((3, 2)), np.ones((2, 2)), precision=3)


def test_mfma_f64_rate_probe(ctx):
    """The attainable float64 MFMA rate the bench reports beside the published peak: a
    positive rate that does not exceed the published 78.6 TFLOP/s (the probe's flop count
    is exact, so a rate above the peak would mean a wrong count or timing)."""
    r = ctx.mfma_f64_rate()
    assert 1.0 < r <= 78.6 * 1.02, r
