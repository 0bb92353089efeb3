"""Checks at the size the benchmark times: L=48, N=24, rank cap 512, m_zip 512, simultaneous
truncation.  A dense oracle vector would have 2^48 entries, so these are properties that
hold at any size and outputs the oracle evaluates one at a time:
- every Rayleigh quotient is >= 1 (gamma makes lambda_1(H_gamma) >= 1) and each Ritz value
  is not above the Rayleigh quotient of its step;
- the truncation guarantee ||x - trunc_eps(x)|| <= eps, from three overlaps;
- the sandwich is symmetric, <a|H|b> = <b|H|a>, between two different states;
- overlaps <det|psi> with sampled determinants equal the matrix product of the downloaded
  MPS along each determinant (oracle.mps.amplitude)."""
import math

import numpy as np
import pytest

from oracle import mps as omps
from synth import make_problem

pytestmark = pytest.mark.gpu

native = pytest.importorskip("paper_2604_16118_amd.native")

L, N, CAP = 48, 24, 512


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = native.Context(0)
    p = make_problem("decayed", L, N, 0)
    ctx.set_hamiltonian(p.h, p.v, N, p.gamma)
    _, hist, psi = ctx.run(rank_cap=CAP, max_iter=4, tau=0.0, c=0.5, delta=10.0, m_zip=CAP, truncation=1)
    ctx.set_truncation(1)
    yield ctx, p, hist, psi
    ctx.mps_free(psi)
    ctx.close()


def test_rayleigh_quotients_and_ritz_values(full):
    ctx, p, hist, psi = full
    assert len(hist) == 4
    for r in hist:
        assert r["lam"] >= 1.0
        assert r["lam_star"] <= r["lam"] * (1 + 1e-12)
    assert hist[-1]["E"] < hist[0]["E"]
    assert max(r["max_rank"] for r in hist) == CAP


def test_truncation_guarantee(full):
    ctx, p, hist, psi = full
    nx = ctx.dot(psi, psi)
    eps = 1e-3 * math.sqrt(nx)
    y, cap_bound = ctx.round(psi, eps, CAP)
    try:
        d2 = nx + ctx.dot(y, y) - 2.0 * ctx.dot(psi, y)
        assert not cap_bound
        assert d2 <= eps * eps * (1 + 1e-6) + 1e-12 * nx
        rho_x, _ = ctx.mps_layout(psi)
        rho_y, _ = ctx.mps_layout(y)
        assert rho_y.sum() < rho_x.sum()  # the tolerance removed something
    finally:
        ctx.mps_free(y)


def test_sandwich_is_symmetric(full):
    ctx, p, hist, psi = full
    y, _ = ctx.round(psi, 1e-2 * math.sqrt(ctx.dot(psi, psi)), CAP)
    try:
        a, b = ctx.expect_h(psi, y), ctx.expect_h(y, psi)
        assert abs(a - b) <= 1e-10 * abs(a)
    finally:
        ctx.mps_free(y)


def test_sampled_amplitudes(full):
    ctx, p, hist, psi = full
    rho, data = ctx.mps_download(psi)
    occ0 = sorted(np.argsort(np.diag(p.h), kind="stable")[:N].tolist())
    virt = [a for a in range(L) if a not in occ0]
    samples = [occ0,
               sorted([o for o in occ0 if o != occ0[-1]] + [virt[0]]),
               sorted([o for o in occ0 if o != occ0[-2]] + [virt[1]]),
               sorted([o for o in occ0 if o not in occ0[-2:]] + virt[:2])]
    scale = math.sqrt(ctx.dot(psi, psi))
    for occ in samples:
        cfg = sum(1 << i for i in occ)
        want = omps.amplitude(L, N, rho, data, cfg)
        d = ctx.mps_determinant(occ)
        try:
            got = ctx.dot(d, psi)
        finally:
            ctx.mps_free(d)
        assert abs(got - want) <= 1e-12 * scale + 1e-10 * abs(want), (occ, got, want)
