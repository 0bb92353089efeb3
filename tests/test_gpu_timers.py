"""Kernel-class timing switch (pv_set_timer_mask): an untimed class records no launches and
the results do not depend on which classes are timed."""
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


def test_untimed_class_accumulates_nothing(ctx):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((150, 70))
    B = rng.standard_normal((70, 90))
    ctx.timers_reset()
    ctx.set_timed_classes(["jacobi_eig_f64"])
    C1 = ctx.gemm(A, B)
    t = ctx.timers()
    assert t["gemm_f64_mfma"]["calls"] == 0 and t["gemm_f64_mfma"]["ms"] == 0.0
    ctx.set_timed_classes(None)
    C2 = ctx.gemm(A, B)
    t = ctx.timers()
    assert t["gemm_f64_mfma"]["calls"] >= 1 and t["gemm_f64_mfma"]["ms"] > 0.0
    assert np.array_equal(C1, C2)
    np.testing.assert_allclose(C1, A @ B, rtol=1e-12, atol=1e-12)


def test_unknown_class_is_rejected(ctx):
    with pytest.raises(ValueError):
        ctx.set_timed_classes(["no_such_class"])


def test_sampled_timing_counts_for_the_launches_it_stands_for(ctx):
    """One-in-eight sampled timing: every timed launch counts for eight, the selection is
    deterministic (the same launches after a reset) and results do not depend on it."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((70, 40))
    B = rng.standard_normal((40, 30))
    counts = []
    for _ in range(2):
        ctx.timers_reset()
        ctx.set_timed_classes(["gemm_f64_mfma"])
        ctx.set_timer_sampling(["gemm_f64_mfma"], 8)
        outs = [ctx.gemm(A, B) for _ in range(64)]
        t = ctx.timers()["gemm_f64_mfma"]
        counts.append(t["calls"])
        assert t["calls"] % 8 == 0 and 8 <= t["calls"] <= 160
        assert t["ms"] > 0.0
        assert all(np.array_equal(o, outs[0]) for o in outs)
    ctx.set_timer_sampling(None)
    ctx.set_timed_classes(None)
    assert counts[0] == counts[1]
    with pytest.raises(Exception):
        ctx.set_timer_sampling(["gemm_f64_mfma"], 0)
