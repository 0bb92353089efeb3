"""GPU z-form Algorithm 2 (pv_run_zform) against the oracle's (oracle.zform.run_z): energy of
every iteration within 1e-10 (relative), with the same tolerance reductions and cap flags,
and its equality with the psi-form of pv_run when nothing is truncated."""
import pytest

from oracle import fock, pinvit, zform
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


def _compare(ctx, kind, L, N, seed, cap, iters, truncation=0, tol=1e-10):
    p = make_problem(kind, L, N, seed)
    w = fock.lowest_eigs(p.h, p.v, N, p.gamma, k=2)
    delta = w[1] / (w[1] - w[0])
    prm = pinvit.Params(cap=cap, max_iter=iters, tau=1e-12, c=0.5, delta=delta,
                        truncation="parallel" if truncation else "sequential")
    _, hist_o, _ = zform.run_z(p.h, p.v, N, p.gamma, prm)
    ctx.set_hamiltonian(p.h, p.v, N, p.gamma)
    _, hist_g, x = ctx.run_zform(rank_cap=cap, max_iter=iters, tau=1e-12, c=0.5, delta=delta, truncation=truncation)
    ctx.mps_free(x)
    assert len(hist_g) == len(hist_o)
    for a, b in zip(hist_g, hist_o):
        assert abs(a["E"] - b["E"]) <= tol * abs(b["E"]), (a["E"], b["E"])
        assert a["retries"] == b["retries"]
        assert a["cap_bound"] == b["cap_bound"]
        assert a["rho"] == pytest.approx(b["rho"], rel=1e-6)
        assert a["lam"] >= w[0] - 1e-12
    return hist_g


def test_zform_matches_oracle(ctx):
    _compare(ctx, "decayed", 8, 4, 0, 64, 6)


def test_zform_capped_matches_oracle(ctx):
    _compare(ctx, "decayed", 8, 4, 1, 6, 5)


def test_zform_three_particles(ctx):
    _compare(ctx, "dense", 7, 3, 2, 32, 5)


def test_zform_parallel_truncation_matches_oracle(ctx):
    _compare(ctx, "decayed", 8, 4, 3, 64, 4, truncation=1)


def test_zform_equals_psi_form_without_truncation(ctx):
    p = make_problem("decayed", 8, 4, 0)
    ctx.set_hamiltonian(p.h, p.v, 4, p.gamma)
    kw = dict(rank_cap=64, max_iter=6, tau=1e-12, c=0.5, delta=10.0, eps_num=1e-13, t_eig=1e-13)
    _, hz, x = ctx.run_zform(**kw)
    _, hp, psi = ctx.run(**kw)
    ctx.mps_free(x)
    ctx.mps_free(psi)
    assert len(hz) == len(hp)
    for a, b in zip(hz, hp):
        assert abs(a["E"] - b["E"]) <= 1e-10 * abs(b["E"])


def test_zform_rejects_float32(ctx):
    p = make_problem("decayed", 6, 3, 0)
    ctx.set_hamiltonian(p.h, p.v, 3, p.gamma)
    with pytest.raises(native.PvError):
        ctx.run_zform(rank_cap=8, max_iter=2, precision=1)
