"""GEMM tile shapes and their autotuner (pv_set_gemm_tiles, pv_gemm_tune_table): the two
float64 tile shapes form every element of C by the same chain of MFMA products, so they
must agree bit for bit (and with NumPy to rounding); the online autotuner must time both
shapes, decide every key it explored, and leave every result, down to whole Algorithm 2
runs, bit-identical to the fixed rule's."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

native = pytest.importorskip("paper_2604_16118_amd.native")
from synth import make_problem  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = native.Context(0)
    yield c
    c.set_gemm_tiles("rule")
    c.close()


# one tile to thousands, split-K (K = 5000 on few tiles), ragged edges
SHAPES = [(100, 90, 37), (1100, 1030, 70), (200, 2000, 45), (120, 96, 5000), (65, 129, 17),
          (1, 1, 1), (300, 5000, 19)]


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K", SHAPES)
def test_tile_shapes_agree_bit_for_bit(ctx, M, N, K, ta, tb):
    rng = np.random.default_rng(M + 3 * N + 7 * K + ta)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    out = {}
    for mode in ("small", "large", "rule"):
        ctx.set_gemm_tiles(mode)
        out[mode] = ctx.gemm(A, B, C0, ta=ta, tb=tb, alpha=0.75, beta=-1.5)
    ctx.set_gemm_tiles("rule")
    assert np.array_equal(out["small"], out["large"])
    assert np.array_equal(out["rule"], out["large"])
    ref = 0.75 * (A.T if ta else A) @ (B.T if tb else B) - 1.5 * C0
    tol = 1e-14 * K * np.abs(A).max() * np.abs(B).max() + 1e-15 * np.abs(ref).max()
    assert np.abs(out["large"] - ref).max() <= tol


def test_autotuner_decides_and_keeps_bits(ctx):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((700, 64))
    B = rng.standard_normal((64, 600))
    ctx.set_gemm_tiles("rule")
    want = ctx.gemm(A, B)
    native.gemm_tune_clear()
    assert native.gemm_tune_table() == []
    ctx.set_gemm_tiles("tune")
    for _ in range(10):  # 8 exploration launches (4 per shape), then the decided shape
        assert np.array_equal(ctx.gemm(A, B), want)
    rows = native.gemm_tune_table()
    assert len(rows) == 1
    r = rows[0]
    # 700 x 600 is 11 x 10 = 110 tiles of 64 x 64 (bucket 6), K = 64 (bucket 6)
    assert (r["prec"], r["tiles_log2"], r["k_log2"]) == (0, 6, 6)
    assert r["n64"] == 4 and r["n32"] == 4
    assert r["choice"] in (0, 1)
    assert r["tflops64"] > 0 and r["tflops32"] > 0
    faster = 1 if r["tflops32"] > r["tflops64"] else 0
    assert r["choice"] == faster
    ctx.set_gemm_tiles("table")
    assert np.array_equal(ctx.gemm(A, B), want)
    assert native.gemm_tune_table()[0]["n64"] == 4  # no further exploration
    ctx.set_gemm_tiles("rule")


def test_tuned_run_equals_rule_run(ctx):
    """Algorithm 2 at L=12 (mode 1, binding m_zip): the online tuner explores during the
    run and the energies, residual norms and ranks stay bit-identical to the rule's."""
    p = make_problem("decayed", 12, 6, 2)
    ctx.set_hamiltonian(p.h, p.v, 6, p.gamma)
    kw = dict(rank_cap=32, max_iter=4, tau=0.0, truncation=1, m_zip=32)
    ctx.set_gemm_tiles("rule")
    r0, h0 = ctx.run(**kw)[:2]
    native.gemm_tune_clear()
    ctx.set_gemm_tiles("tune")
    r1, h1 = ctx.run(**kw)[:2]
    ctx.set_gemm_tiles("rule")
    assert r1["energy"] == r0["energy"] and r1["iterations"] == r0["iterations"]
    assert [h["E"] for h in h1] == [h["E"] for h in h0]
    assert [h["rho"] for h in h1] == [h["rho"] for h in h0]
    rows = native.gemm_tune_table()
    assert rows and all(r["n64"] + r["n32"] >= 1 for r in rows)


def test_bad_mode_is_rejected(ctx):
    with pytest.raises(native.PvError):
        ctx.set_gemm_tiles(7)
