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
