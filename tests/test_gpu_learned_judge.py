"""Per-step judge of a corrected S against the plain S (pv_set_learned_judge): from the
same start, a judged iteration's Ritz value is the lower of its two candidates. When the
corrected S wins, the judged iteration equals the corrected-only iteration bit for bit.
When the plain S wins, its Ritz value is strictly lower. The iteration's own lambda and
rho never depend on the judge, the correction stays in force after a judged run, and with
no correction the judge does nothing."""
import numpy as np
import pytest

from oracle import precond
from synth import make_problem

pytestmark = pytest.mark.gpu

native = pytest.importorskip("paper_2604_16118_amd.native")

L, N = 8, 4
RUN = dict(rank_cap=24, tau=0.0, truncation=0)


@pytest.fixture(scope="module")
def prob():
    return make_problem("decayed", L, N, 0)


@pytest.fixture(scope="module")
def ctx(prob):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = native.Context(0)
    c.set_hamiltonian(prob.h, prob.v, N, prob.gamma)
    yield c
    c.set_learned_judge(False)
    c.set_correction(None)
    c.close()


def _tables(p):
    """Corrections Delta[i, k] (site i, k particles before it): zero, a mild smooth one,
    and a harmful one that distorts theta by up to 90% while keeping it positive."""
    th = precond.theta(p.h, p.v, N, p.gamma)
    ks = np.arange(N + 1)
    mild = 0.1 * th[:, None] * np.cos(0.7 * np.arange(L)[:, None] + 0.3 * ks[None, :])
    harm = np.where((np.arange(L) % 2 == 0)[:, None], 0.9, -0.5) * th[:, None] * np.ones((1, N + 1))
    return {"zero": np.zeros((L, N + 1)), "mild": mild, "harmful": harm}


def _run(ctx, iters, judge):
    ctx.set_learned_judge(judge)
    try:
        _, hist, psi = ctx.run(max_iter=iters, **RUN)
        ctx.mps_free(psi)
        return hist, ctx.learned_judge_counts()
    finally:
        ctx.set_learned_judge(False)


@pytest.mark.parametrize("name", ["zero", "mild", "harmful"])
def test_one_judged_step_takes_the_lower_ritz_value(ctx, prob, name):
    corr = _tables(prob)[name]
    ctx.set_correction(corr)
    try:
        info = ctx.precond_info()
        hc, cc = _run(ctx, 1, False)
        hj, cj = _run(ctx, 1, True)
        assert ctx.precond_info() == info  # the corrected S is in force again
    finally:
        ctx.set_correction(None)
    assert cc == (0, 0)
    assert sum(cj) == 1
    a, b = hc[0], hj[0]
    assert b["E"] == a["E"] and b["rho"] == a["rho"] and b["lam"] == a["lam"]
    if cj == (0, 1):  # the corrected S won: the same step
        assert b["lam_star"] == a["lam_star"]
        assert b["eta_psi"] == a["eta_psi"]
    else:  # the plain S won
        assert b["lam_star"] < a["lam_star"]


def test_judged_runs_never_take_a_worse_first_step_and_count_every_step(ctx, prob):
    ctx.set_correction(_tables(prob)["harmful"])
    try:
        hc, _ = _run(ctx, 6, False)
        hj, cj = _run(ctx, 6, True)
    finally:
        ctx.set_correction(None)
    assert sum(cj) == len(hj)
    assert hj[0]["lam_star"] <= hc[0]["lam_star"]
    assert all(np.isfinite(r["E"]) for r in hj)


def test_judge_without_correction_does_nothing(ctx):
    hp, _ = _run(ctx, 3, False)
    hj, cj = _run(ctx, 3, True)
    assert cj == (0, 0)
    assert [r["E"] for r in hj] == [r["E"] for r in hp]
    assert [r["lam_star"] for r in hj] == [r["lam_star"] for r in hp]


def test_judge_rejects_bad_arguments(ctx):
    L_ = native.lib()
    assert L_.pv_set_learned_judge(ctx._p, 2) == -1
    assert L_.pv_set_learned_judge(None, 1) == -1
