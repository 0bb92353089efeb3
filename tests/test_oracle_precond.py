"""Pins of the preconditioner helpers against printed values and closed forms."""
import math

import numpy as np
import pytest

from oracle import bounds, fock, precond
from synth import make_problem


def test_term_counts_reproduce_printed_values(golden):
    for T, ns, *_ in golden("expsum_terms.txt"):
        h, mp, mm = precond.expsum_params(0.1, float(T))
        assert mp - mm + 1 == int(ns)


@pytest.mark.parametrize("c0,T", [(0.1, 9.53), (0.1, 186.52), (0.05, 1000.0), (0.3, 50.0)])
def test_exponential_sum_relative_error(c0, T):
    # eq. Srelerror: |t^-1/2 - S(t)| <= c0 t^-1/2 on [1, T]
    h, mp, mm = precond.expsum_params(c0, T)
    t = np.concatenate([np.linspace(1.0, T, 4001), np.geomspace(1.0, T, 4001)])
    err = np.abs(1.0 / np.sqrt(t) - precond.expsum(t, h, mp, mm)) * np.sqrt(t)
    assert err.max() <= c0


def test_printed_spectral_constants(golden):
    for lo, up, c_pr, en_pr, *_ in golden("spectral_constants.txt"):
        c = precond.c_const(0.0, float(lo), float(up))
        assert round(c, 2) == float(c_pr)
        assert abs(0.5 * (1 - c) - float(en_pr)) <= 0.0051  # printed to two digits


def test_printed_gap_constants(golden):
    for l1, l2, d_pr, *_ in golden("gap_delta.txt"):
        assert round(bounds.gap_delta(float(l1), float(l2)), 4) == float(d_pr)


def test_theta_sum_equals_determinant_energy():
    # for orbitals 1..N the window of theta_i is exactly the occupied set, so
    # sum_{i<=N} theta_i = <e|H + gamma|e> for the determinant e on 1..N (Section 7.1.1)
    p = make_problem("dense", 8, 4, 0)
    th = precond.theta(p.h, p.v, 4, p.gamma)
    e = fock.determinant(8, range(4))
    assert th[:4].sum() == pytest.approx(e @ fock.apply_h(p.h, p.v, e, p.gamma), abs=1e-12)


def test_s_diagonal_equals_scaled_expsum_of_d():
    # Section 4.3 product form == alpha_0 S(D/t_min) (Cor. lrprecond, eq. Sdef)
    p = make_problem("dense", 8, 4, 0)
    pre = precond.Preconditioner(p.h, p.v, 4, p.gamma)
    basis = fock.sector_basis(8, 4)
    dsum = np.zeros(1 << 8)
    idx = np.arange(1 << 8)
    for i in range(8):
        dsum += ((idx >> i) & 1) * pre.th[i]
    want = pre.a0 * precond.expsum(dsum[basis] / pre.t_min, pre.h, pre.m_plus, pre.m_minus)
    got = sum(pre.diagonals())[basis]
    assert np.allclose(got, want, rtol=1e-13)
    assert got.max() <= pre.s_max * (1 + 1e-13) and got.min() >= pre.s_min * (1 - 1e-13)


def test_preconditioned_operator_spectral_equivalence():
    # Cor. lrprecond, eq. specequivA with exact C_lower, C_upper of D^-1/2 H D^-1/2
    L, N = 8, 4
    p = make_problem("dense", L, N, 0)
    th = precond.theta(p.h, p.v, N, p.gamma)
    basis = fock.sector_basis(L, N)
    d = np.array([sum(th[i] for i in range(L) if b >> i & 1) for b in basis])
    H = fock.sector_hamiltonian(p.h, p.v, N, p.gamma)
    w = np.linalg.eigvalsh(H / np.sqrt(np.outer(d, d)))
    cl, cu = w[0], w[-1]
    c0 = 0.1
    pre = precond.Preconditioner(p.h, p.v, N, p.gamma, c0, cl, cu)
    S = sum(pre.diagonals())[basis]
    A = S[:, None] * H * S[None, :]
    wa = np.linalg.eigvalsh(A)
    c = precond.c_const(c0, cl, cu)
    assert wa[0] >= 1 - c - 1e-12 and wa[-1] <= 1 + c + 1e-12


def test_sorted_sum_meets_tolerance():
    L, N = 8, 4
    p = make_problem("dense", L, N, 1)
    pre = precond.Preconditioner(p.h, p.v, N, p.gamma)
    x = np.zeros(1 << L)
    x[fock.sector_basis(L, N)] = np.random.default_rng(0).standard_normal(70)
    exact = pre.apply_exact(x)
    for eta in (1e-1, 1e-3, 1e-6):
        y, cb, nr, _ = precond.apply_sorted(pre, x, eta, 1000, N)
        assert not cb
        assert np.linalg.norm(y - exact) <= eta * (1 + 1e-12)
