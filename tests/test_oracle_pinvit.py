"""Invariants of the oracle's Algorithm 2 run against exact diagonalisation."""
import math

import numpy as np
import pytest

from oracle import fock, pinvit
from synth import make_problem


def _exact(p, N):
    w = fock.lowest_eigs(p.h, p.v, N, p.gamma, k=2)
    return w[0], w[1] / (w[1] - w[0])


def test_config_small_dense_invariants():
    # L=8, N=4, dense integrals seed 0, cap 16, 20 iterations
    p = make_problem("dense", 8, 4, 0)
    l1, delta = _exact(p, 4)
    prm = pinvit.Params(cap=16, max_iter=20, tau=1e-12, c=0.5, delta=delta)
    psi, hist, _ = pinvit.run(p.h, p.v, 4, p.gamma, prm)
    lams = [r["lam"] for r in hist]
    assert all(l >= l1 - 1e-12 for l in lams)                      # variational (eq. rayleigh1)
    assert all(b <= a + 1e-12 for a, b in zip(lams, lams[1:]))       # monotone decrease
    for a, b in zip(hist, hist[1:]):                                 # eq. modqcond
        if not a["cap_bound"] and not a.get("cap_bound_update"):
            assert b["lam"] <= a["lam_star"] + 0.5 * (a["lam"] - a["lam_star"]) + 1e-12
    # the a-posteriori eigenvalue bound holds at every iteration where it is defined
    from oracle import bounds
    for r in hist:
        bnd = bounds.rel_eig_bound(r["rho"], delta)
        if r["rho"] ** 2 <= 1 / (4 * delta * (delta - 1)) and not math.isnan(bnd):
            assert (r["lam"] - l1) / l1 <= bnd * (1 + 1e-9)


@pytest.mark.slow
def test_extended_run_reaches_exact_ground_energy():
    p = make_problem("dense", 8, 4, 0)
    l1, delta = _exact(p, 4)
    prm = pinvit.Params(cap=16, max_iter=150, tau=1e-7, c=0.5, delta=delta)
    psi, hist, _ = pinvit.run(p.h, p.v, 4, p.gamma, prm)
    assert hist[-1].get("stop")
    assert abs(hist[-1]["lam"] - l1) <= 1e-10 * abs(hist[-1]["E"])


def test_noninteracting_limit():
    p = make_problem("decayed", 8, 3, 2)
    v = np.zeros_like(p.v)
    e0 = np.sort(np.linalg.eigvalsh(p.h))[:3].sum()
    prm = pinvit.Params(cap=20, max_iter=200, tau=1e-7, c=0.5, delta=10.0)
    psi, hist, _ = pinvit.run(p.h, v, 3, p.gamma, prm)
    assert abs(hist[-1]["E"] - e0) <= 1e-9 * abs(e0)



def test_outer_iteration_against_exact_diagonalisation():
    """Algorithm 3: the returned eigenvalue meets |lambda - lambda_1| < lambda_1 tol (its
    stated output guarantee), the relative bound of eq. releigerr bounds the true error at
    every outer step, every outer truncation stays within its tolerance, eta halves, and
    the inner tolerance is eta^m / (2 (1 + (1+alpha) kappa))."""
    from oracle import bounds
    p = make_problem("dense", 8, 4, 0)
    l1, delta = _exact(p, 4)
    prm = pinvit.Params(cap=16, max_iter=40, c=0.5, delta=delta)
    alpha, tol = 1.0, 1e-9
    psi, outer = pinvit.run_outer(p.h, p.v, 4, p.gamma, prm, alpha=alpha, tol=tol, max_outer=12)
    assert outer[-1].get("stop")
    lam = outer[-1]["lam"]
    assert abs(lam - l1) < l1 * tol
    kappa = math.sqrt(3.0) * math.sqrt(7.0)            # eq. kappadef with c = 1/2, K = 8
    theta = 2 * kappa / (2 * (1 + 2 * kappa))
    assert outer[0]["eta"] == pytest.approx(1 / (2 * theta), rel=1e-15)
    for a, b in zip(outer, outer[1:]):
        assert b["eta"] == pytest.approx(0.5 * a["eta"], rel=1e-15)
    for r in outer:
        assert r["tau"] == pytest.approx(r["eta"] / (2 * (1 + 2 * kappa)), rel=1e-15)
        if not math.isnan(r["rel_bound"]):
            assert (r["lam"] - l1) / l1 <= r["rel_bound"] * (1 + 1e-9)
        if "trunc_eps" in r:
            assert r["trunc_err"] <= r["trunc_eps"] * (1 + 1e-9)
    # the normalised result is close to the ground state
    w, V = np.linalg.eigh(fock.sector_hamiltonian(p.h, p.v, 4, p.gamma))
    u = np.zeros_like(psi)
    u[fock.sector_basis(8, 4)] = V[:, 0]
    assert abs(abs(float(psi @ u)) - 1.0) <= 1e-6
