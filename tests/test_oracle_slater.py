"""Pins of the Slater-determinant matrix elements (oracle/slater.py) against the
Hamiltonian applied to dense vectors by its definition (oracle/fock.py)."""
import numpy as np
import pytest

from oracle import fock, slater
from synth import make_problem


@pytest.mark.parametrize("kind,L,N,seed", [("dense", 8, 4, 0), ("decayed", 8, 3, 2), ("dense", 7, 2, 5)])
def test_elements_equal_the_sector_hamiltonian(kind, L, N, seed):
    p = make_problem(kind, L, N, seed)
    H = fock.sector_hamiltonian(p.h, p.v, N, p.gamma)
    basis = fock.sector_basis(L, N)
    E = np.array([[slater.element(p.h, p.v, p.gamma, int(a), int(b)) for b in basis] for a in basis])
    assert np.abs(E - H).max() <= 1e-13 * np.abs(H).max()


def test_elements_vanish_beyond_double_excitations_and_are_symmetric():
    L, N = 10, 5
    p = make_problem("decayed", L, N, 1)
    rng = np.random.default_rng(0)
    basis = fock.sector_basis(L, N)
    for _ in range(200):
        a, b = (int(x) for x in rng.choice(basis, 2))
        e = slater.element(p.h, p.v, p.gamma, a, b)
        assert e == pytest.approx(slater.element(p.h, p.v, p.gamma, b, a), abs=1e-14)
        if bin(a ^ b).count("1") > 4:
            assert e == 0.0
        else:
            x = fock.determinant(L, [i for i in range(L) if b >> i & 1])
            y = fock.apply_h(p.h, p.v, x, p.gamma)
            assert e == pytest.approx(y[a], abs=1e-13)


def test_excitation_lists():
    L, b = 6, 0b000111
    s = slater.single_excitations(b, L)
    d = slater.double_excitations(b, L)
    assert len(s) == 9 and len(set(s)) == 9 and all(bin(x).count("1") == 3 and bin(x ^ b).count("1") == 2 for x in s)
    assert len(d) == 9 and all(bin(x ^ b).count("1") == 4 for x in d)
