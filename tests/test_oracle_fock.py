"""Pins of the oracle's Fock-space layer against the paper's definitions and textbook cases."""
import math

import numpy as np
import pytest

from oracle import fock
from synth import make_problem, random_dense


def test_bitstring_operators_match_kronecker_definition():
    L = 5
    ops = fock.kron_ops(L)
    eye = np.eye(1 << L)
    for i in range(L):
        assert np.array_equal(fock.annihilate(eye, i), ops[i])
        assert np.array_equal(fock.create(eye, i), ops[i].T)


def test_anticommutation_relations():
    # Section 1.1, eq. anticomm, on the literal Kronecker matrices and the bit-string maps
    L = 5
    ops = fock.kron_ops(L)
    eye = np.eye(1 << L)
    for i in range(L):
        for j in range(L):
            ac = ops[i] @ ops[j].T + ops[j].T @ ops[i]
            assert np.array_equal(ac, eye * (i == j))
            assert not np.any(ops[i] @ ops[j] + ops[j] @ ops[i])
            x = np.random.default_rng(i * L + j).standard_normal(1 << L)
            y = fock.annihilate(fock.create(x, j), i) + fock.create(fock.annihilate(x, i), j)
            assert np.allclose(y, x * (i == j), atol=0)


def test_apply_h_matches_kronecker_sum():
    L = 5
    h, v = random_dense(L, 3)
    # break the 8-fold symmetry too: apply_h must follow eq. hamil for any coefficients
    v = v + 0.01 * np.random.default_rng(1).standard_normal(v.shape)
    ops = fock.kron_ops(L)
    H = np.zeros((1 << L, 1 << L))
    for i in range(L):
        for j in range(L):
            H += h[i, j] * ops[i].T @ ops[j]
            for k in range(L):
                for l in range(L):
                    H += v[i, j, k, l] * ops[i].T @ ops[j].T @ ops[k] @ ops[l]
    x = np.random.default_rng(0).standard_normal((1 << L, 3))
    assert np.allclose(fock.apply_h(h, v, x, 0.7), H @ x + 0.7 * x, rtol=0, atol=1e-12)


def test_hamiltonian_hermitian_and_number_conserving():
    p = make_problem("dense", 8, 4, 0)
    H = fock.sector_hamiltonian(p.h, p.v, 4)
    assert np.allclose(H, H.T, atol=1e-12)
    x = np.zeros(1 << 8)
    x[fock.sector_basis(8, 4)] = np.random.default_rng(0).standard_normal(70)
    y = fock.apply_h(p.h, p.v, x)
    assert np.allclose(fock.number_op(y), 4 * y, atol=1e-12)
    outside = np.ones(1 << 8, bool)
    outside[fock.sector_basis(8, 4)] = False
    assert np.max(np.abs(y[outside])) == 0.0


def test_sector_dimension():
    for L, N in [(8, 4), (10, 3), (6, 6), (6, 0)]:
        assert len(fock.sector_basis(L, N)) == math.comb(L, N)


def test_noninteracting_ground_energy_is_sum_of_orbital_energies():
    h, _ = random_dense(8, 5)
    v = np.zeros((8,) * 4)
    for N in (1, 3, 4):
        e = fock.lowest_eigs(h, v, N, k=1)[0]
        assert e == pytest.approx(np.sort(np.linalg.eigvalsh(h))[:N].sum(), abs=1e-12)


def test_one_particle_sector_ignores_two_body_part():
    h, v = random_dense(7, 2)
    assert fock.lowest_eigs(h, v, 1, k=1)[0] == pytest.approx(np.linalg.eigvalsh(h)[0], abs=1e-12)


def test_two_particle_sector_matches_textbook_pair_matrix():
    L = 7
    h, v = random_dense(L, 4)
    w = v - v.transpose(1, 0, 2, 3) - v.transpose(0, 1, 3, 2) + v.transpose(1, 0, 3, 2)
    pairs = [(i, j) for i in range(L) for j in range(i + 1, L)]
    M = np.zeros((len(pairs), len(pairs)))
    d = lambda a, b: float(a == b)  # noqa: E731
    for a, (i, j) in enumerate(pairs):
        for b, (k, l) in enumerate(pairs):
            M[a, b] = (h[i, k] * d(j, l) - h[j, k] * d(i, l) - h[i, l] * d(j, k)
                       + h[j, l] * d(i, k) - w[i, j, k, l])
    assert fock.lowest_eigs(h, v, 2, k=1)[0] == pytest.approx(np.linalg.eigvalsh(M)[0], abs=1e-11)


def test_shift_makes_sector_spectrum_at_least_one():
    p = make_problem("dense", 8, 4, 0)
    assert fock.lowest_eigs(p.h, p.v, 4, p.gamma, k=1)[0] >= 1.0 - 1e-12


@pytest.mark.slow
def test_lanczos_agrees_with_dense_eigh():
    p = make_problem("decayed", 12, 6, 1)
    dense = np.linalg.eigvalsh(fock.sector_hamiltonian(p.h, p.v, 6))[:2]
    from scipy.sparse.linalg import LinearOperator, eigsh
    basis = fock.sector_basis(12, 6)

    def mv(y):
        x = np.zeros(1 << 12)
        x[basis] = y.ravel()
        return fock.apply_h(p.h, p.v, x)[basis]

    w = np.sort(eigsh(LinearOperator((924, 924), matvec=mv, dtype=float), k=2, which="SA",
                      tol=1e-13, return_eigenvectors=False))
    assert np.allclose(w, dense, atol=1e-10)
