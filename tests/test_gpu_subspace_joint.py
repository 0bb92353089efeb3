"""Algorithm 4 with the columns held jointly (Section 6.2) through pv_run_subspace_joint,
against the oracle's joint iteration (oracle/subspace.run_subspace_joint): the D values
of every iteration, retries, cap flags and the final columns, in both truncation modes,
with a cap that holds the summed ranks and with a binding one; one column against
pv_run_subspace."""
import numpy as np
import pytest

from oracle import fock, mps as omps, pinvit, subspace
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


def _columns(ctx, h, L, N, D):
    rho, data = ctx.mps_download(h)
    assert rho[L][N] == D
    blk = omps.unpack(L, N, rho, data)
    cols = []
    for i in range(D):
        sel = {}
        for (k, n, kind), b in blk.items():
            sel[(k, n, kind)] = b[:, i:i + 1] if k == L else b
        r1 = np.array(rho)
        r1[L][N] = 1
        flat = np.concatenate([sel[(k, n, kind)].T.reshape(-1) for k, n, kind, _, _ in omps.block_shapes(L, N, r1)])
        cols.append(omps.to_dense(L, N, r1, flat))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("D,cap,mode,tol", [(2, 64, "sequential", 1e-10), (3, 64, "sequential", 1e-10),
                                            (3, 20, "sequential", 1e-10), (2, 64, "parallel", 1e-6)])
def test_joint_subspace_matches_oracle(ctx, D, cap, mode, tol):
    L, N = 8, 4
    p = make_problem("dense", L, N, 0)
    w = fock.lowest_eigs(p.h, p.v, N, p.gamma, k=D + 1)
    delta = w[D] / (w[D] - w[0])
    iters = 10
    prm = pinvit.Params(cap=cap, max_iter=iters, tau=1e-12, c=0.5, delta=delta, truncation=mode)
    X_o, hist_o, _ = subspace.run_subspace_joint(p.h, p.v, N, p.gamma, prm, D)
    ctx.set_hamiltonian(p.h, p.v, N, p.gamma)
    res, hist_g, h = ctx.run_subspace_joint(D, rank_cap=cap, max_iter=iters, tau=1e-12, c=0.5, delta=delta,
                                            truncation=0 if mode == "sequential" else 1)
    assert len(hist_g) == len(hist_o)
    for a, b in zip(hist_g, hist_o):
        assert np.all(np.abs(a["lam"] - b["lam"]) <= tol * np.abs(b["lam"])), (a["lam"], b["lam"])
        assert np.all(a["lam"] >= w[:D] - 1e-10)
        if tol <= 1e-10:
            assert a["retries"] == b["retries"]
            assert a["cap_bound"] == b["cap_bound"]
    if tol <= 1e-10:
        X = _columns(ctx, h, L, N, D)
        for i in range(D):
            ov = abs(X[:, i] @ X_o[:, i]) / (np.linalg.norm(X[:, i]) * np.linalg.norm(X_o[:, i]))
            assert abs(ov - 1) <= 1e-8
    ctx.mps_free(h)


def test_joint_one_column_equals_the_separate_iteration(ctx):
    L, N = 8, 4
    p = make_problem("dense", L, N, 2)
    ctx.set_hamiltonian(p.h, p.v, N, p.gamma)
    kw = dict(rank_cap=16, max_iter=8, tau=0.0, c=0.5, delta=10.0)
    _, hj, hh = ctx.run_subspace_joint(1, **kw)
    _, hs, hs_h = ctx.run_subspace(1, **kw)
    assert len(hj) == len(hs)
    for a, b in zip(hj, hs):
        assert abs(a["lam"][0] - b["lam"][0]) <= 1e-12 * b["lam"][0]
    ctx.mps_free(hh)
    for x in hs_h:
        ctx.mps_free(x)


def test_joint_start_from_a_given_joint_mps(ctx):
    """A start of D columns given as one joint MPS (pv_mps_create with rho[L][N] = D) runs
    as the oracle's iteration from the same columns."""
    L, N, D = 8, 4, 2
    p = make_problem("dense", L, N, 0)
    ctx.set_hamiltonian(p.h, p.v, N, p.gamma)
    dets = subspace.start_determinants(p.h, N, D)
    hs = [ctx.mps_determinant(o) for o in dets]
    _, _, hjoint = ctx.run_subspace_joint(D, rank_cap=64, max_iter=1, tau=0.0, c=0.5, delta=10.0)
    rho, data = ctx.mps_download(hjoint)
    h2 = ctx.mps_create(rho, data)
    X0 = _columns(ctx, h2, L, N, D)
    prm = pinvit.Params(cap=64, max_iter=4, tau=0.0, c=0.5, delta=10.0)
    _, hist_o, _ = subspace.run_subspace_joint(p.h, p.v, N, p.gamma, prm, D, X0=X0)
    _, hist_g, h3 = ctx.run_subspace_joint(D, start=h2, rank_cap=64, max_iter=4, tau=0.0, c=0.5, delta=10.0)
    for a, b in zip(hist_g, hist_o):
        assert np.all(np.abs(a["lam"] - b["lam"]) <= 1e-10 * np.abs(b["lam"]))
    for x in hs + [hjoint, h2, h3]:
        ctx.mps_free(x)
