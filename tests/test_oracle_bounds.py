"""Pins of the Ritz step and a-posteriori bounds (Section 5.4, Rem. omegamin)."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import bounds, fock, precond
from synth import make_problem


def test_ritz2_matches_generalised_eigh_and_line_search():
    rng = np.random.default_rng(0)
    for _ in range(20):
        B = rng.standard_normal((6, 2))
        H = rng.standard_normal((6, 6))
        H = H @ H.T + 0.1 * np.eye(6)
        hm, mm = B.T @ H @ B, B.T @ B
        lam, v = bounds.ritz2(hm, mm)
        w, V = scipy.linalg.eigh(hm, mm)
        assert lam == pytest.approx(w[0], rel=1e-12)
        assert v @ mm @ v == pytest.approx(1.0, rel=1e-12) and v[0] > 0
        assert np.allclose(hm @ v, lam * mm @ v, atol=1e-10 * np.abs(hm).max())
        # brute force: minimise the Rayleigh quotient along psi + t p
        ts = np.tan(np.linspace(-1.5707, 1.5707, 200001))
        rq = (hm[0, 0] + 2 * ts * hm[0, 1] + ts * ts * hm[1, 1]) / (
            mm[0, 0] + 2 * ts * mm[0, 1] + ts * ts * mm[1, 1])
        assert lam <= rq.min() + 1e-12 and lam == pytest.approx(min(rq.min(), hm[1, 1] / mm[1, 1]), rel=1e-7)


def test_delta_root():
    for rho, q in [(0.1, 0.9), (0.5, 0.99), (0.01, 0.5)]:
        d = bounds.delta_a(rho, q)
        assert 0 < d < 1
        assert math.sqrt(1 - d * d) - rho * d == pytest.approx(q, abs=1e-14)


def _exact_setup(L=8, N=4, seed=0):
    p = make_problem("dense", L, N, seed)
    basis = fock.sector_basis(L, N)
    H = fock.sector_hamiltonian(p.h, p.v, N, p.gamma)
    pre = precond.Preconditioner(p.h, p.v, N, p.gamma)
    S = sum(pre.diagonals())[basis]
    A = S[:, None] * H * S[None, :]
    E = S * S
    w, V = scipy.linalg.eigh(A, np.diag(E))
    return H, S, A, E, w, V


def test_sine_bounds_prop_raylangleb():
    H, S, A, E, w, V = _exact_setup()
    delta = bounds.gap_delta(w[0], w[1])
    u1 = V[:, 0] / math.sqrt(V[:, 0] @ A @ V[:, 0])
    rng = np.random.default_rng(1)
    for scale in (1e-3, 1e-2, 1e-1):
        x = u1 + scale * rng.standard_normal(len(u1))
        lam = (x @ A @ x) / (x @ (E * x))
        cos = (x @ A @ u1) / math.sqrt(x @ A @ x)
        sin2 = 1 - cos * cos
        assert 1 - w[0] / lam <= sin2 * (1 + 1e-9) + 1e-15
        assert sin2 <= delta * (1 - w[0] / lam) * (1 + 1e-9) + 1e-15


def test_eigenvector_error_bound_thm_aposterbound():
    H, S, A, E, w, V = _exact_setup()
    delta = bounds.gap_delta(w[0], w[1])
    u1 = V[:, 0] / math.sqrt(V[:, 0] @ A @ V[:, 0])
    Ainv = np.linalg.inv(A)
    rng = np.random.default_rng(2)
    for scale in (1e-4, 1e-3, 1e-2):
        x = u1 + scale * rng.standard_normal(len(u1))
        lam = (x @ A @ x) / (x @ (E * x))
        r = A @ x - lam * E * x
        rho = math.sqrt(r @ Ainv @ r) / math.sqrt(x @ A @ x)
        xa = x / math.sqrt(x @ A @ x)
        err = math.sqrt((u1 - xa) @ A @ (u1 - xa))
        bnd = bounds.eigvec_error_bound(rho, delta)
        assert err <= bnd * (1 + 1e-9)
        assert (lam - w[0]) / w[0] <= bounds.rel_eig_bound(rho, delta) * (1 + 1e-9)
