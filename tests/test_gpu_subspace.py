"""GPU Algorithm 4 (pv_run_subspace) against the oracle's subspace iteration: the D
Rayleigh quotients of every iteration within 1e-10 (relative), with the same tolerance
reductions and cap decisions, in both truncation modes and with a binding rank cap."""
import numpy as np
import pytest

from oracle import fock, pinvit, subspace
from synth import make_problem

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


def _compare(ctx, kind, L, N, seed, D, cap, iters, truncation=0, tol=1e-10):
    p = make_problem(kind, L, N, seed)
    w = fock.lowest_eigs(p.h, p.v, N, p.gamma, k=D + 1)
    delta = w[1] / (w[1] - w[0])
    prm = pinvit.Params(cap=cap, max_iter=iters, tau=1e-12, c=0.5, delta=delta,
                        truncation="parallel" if truncation else "sequential")
    _, hist_o, _ = subspace.run_subspace(p.h, p.v, N, p.gamma, prm, D)
    ctx.set_hamiltonian(p.h, p.v, N, p.gamma)
    res, hist_g, handles = ctx.run_subspace(D, rank_cap=cap, max_iter=iters, tau=1e-12, c=0.5, delta=delta,
                                            truncation=truncation)
    assert len(hist_g) == len(hist_o)
    for a, b in zip(hist_g, hist_o):
        np.testing.assert_allclose(a["E"], b["E"], rtol=tol, atol=0)
        assert a["retries"] == b["retries"]
        assert a["cap_bound"] == b["cap_bound"]
        np.testing.assert_allclose(a["rho"], b["rho"], rtol=1e-6)
        assert np.all(a["lam"] >= w[:D] - 1e-11 * np.abs(w[:D]))
        if "lam_star" in b:
            np.testing.assert_allclose(a["lam_star"], b["lam_star"], rtol=tol, atol=0)
    assert len(handles) == D
    for h in handles:
        ctx.mps_free(h)
    return hist_g, w


def test_subspace_matches_oracle_exact_ranks(ctx):
    hist, w = _compare(ctx, "decayed", 8, 4, 0, 3, 64, 12)
    # twelve iterations take the first Rayleigh quotient to within 1e-4 of the eigenvalue
    assert 0 <= hist[-1]["lam"][0] - w[0] <= 1e-4 * abs(w[0])
    assert hist[-1]["lam"][0] < hist[0]["lam"][0]


def test_subspace_matches_oracle_capped(ctx):
    hist, _ = _compare(ctx, "decayed", 8, 4, 2, 2, 6, 6)
    assert any(r["cap_bound"] for r in hist)


def test_subspace_three_particles_four_columns(ctx):
    _compare(ctx, "dense", 7, 3, 1, 4, 32, 6)


def test_subspace_parallel_truncation_matches_oracle(ctx):
    _compare(ctx, "decayed", 8, 4, 3, 2, 64, 6, truncation=1)


def test_subspace_one_column_is_pinvit(ctx):
    p = make_problem("decayed", 8, 4, 4)
    ctx.set_hamiltonian(p.h, p.v, 4, p.gamma)
    kw = dict(rank_cap=16, max_iter=6, tau=1e-12, c=0.5, delta=10.0)
    _, h1, hs = ctx.run_subspace(1, **kw)
    _, h2, ha = ctx.run(**kw)
    assert len(h1) == len(h2)
    for a, b in zip(h1, h2):
        assert abs(a["E"][0] - b["E"]) <= 1e-10 * abs(b["E"])
    ctx.mps_free(hs[0])
    ctx.mps_free(ha)


def test_subspace_rejects_bad_arguments(ctx):
    p = make_problem("decayed", 6, 3, 0)
    ctx.set_hamiltonian(p.h, p.v, 3, p.gamma)
    for D in (0, native.SUBSPACE_MAX_D + 1):
        with pytest.raises(ValueError):
            ctx.run_subspace(D, rank_cap=8, max_iter=2)
    with pytest.raises(native.PvError):
        ctx.run_subspace(2, rank_cap=8, max_iter=2, c=1.5)


def test_subspace_continues_from_returned_columns(ctx):
    # starting columns are copied, not consumed; a continuation keeps the Rayleigh quotients
    # above the exact eigenvalues and goes on lowering the first one
    p = make_problem("decayed", 8, 4, 5)
    w = fock.lowest_eigs(p.h, p.v, 4, p.gamma, k=2)
    ctx.set_hamiltonian(p.h, p.v, 4, p.gamma)
    kw = dict(rank_cap=16, tau=1e-12, c=0.5, delta=10.0)
    _, h1, cols = ctx.run_subspace(2, max_iter=3, **kw)
    _, h2, cols2 = ctx.run_subspace(2, starts=cols, max_iter=3, **kw)
    assert h2[-1]["lam"][0] < h1[0]["lam"][0]
    for r in h1 + h2:
        assert np.all(r["lam"] >= w - 1e-11 * np.abs(w))
    for h in cols:  # still valid after the second run
        assert ctx.dot(h, h) > 0
    for h in cols + cols2:
        ctx.mps_free(h)
