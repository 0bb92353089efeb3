"""Pins of the oracle's sector blocks, TT-SVD truncation and MPS contraction."""
import math

import numpy as np
import pytest

from oracle import fock, mps, tt
from synth import layout, random_block_mps, rho_table


def _sector_vector(L, N, seed):
    x = np.zeros(1 << L)
    x[fock.sector_basis(L, N)] = np.random.default_rng(seed).standard_normal(math.comb(L, N))
    return x


def test_block_structure_matches_paper_example(golden):
    # Section 2.3, Example K=5, N=2
    rows = golden("block_example_K5_N2.txt")
    want = {int(r[0]): r[1:] for r in rows}
    L, N = 5, 2
    rho = np.ones((L + 1, N + 1), dtype=int)
    for lay in (mps.block_shapes(L, N, rho), layout(L, N, rho)):
        got = {}
        for k, n, kind, _, _ in lay:
            got.setdefault(k, []).append(("U" if kind == 0 else "O") + str(n))
        assert got == want


def test_sector_sets_and_block_dimensions():
    L, N = 8, 3
    x = _sector_vector(L, N, 0)
    for k in range(L + 1):
        secs = tt.sectors(L, N, k)
        assert secs == [n for n in range(N + 1) if math.comb(k, n) and math.comb(L - k, N - n)]
        if 0 < k < L:
            bl = tt.blocks(x, L, N, k)
            assert sorted(bl) == secs
            assert sum(B.size for _, _, B in bl.values()) == math.comb(L, N)
            for n, (_, _, B) in bl.items():
                assert B.shape == (math.comb(k, n), math.comb(L - k, N - n))


@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-4])
def test_truncation_error_bound(eps):
    L, N = 9, 4
    x = _sector_vector(L, N, 1)
    x /= np.linalg.norm(x)
    y, rho, cb, _, _ = tt.truncate(x, L, N, eps, cap=10 ** 6)
    assert not cb
    assert np.linalg.norm(x - y) <= eps * (1 + 1e-12)
    # exact ranks of the result equal the block table
    r = tt.ranks(y, L, N)
    for k in range(1, L):
        assert {n: c for n, c in r[k].items()} == rho[k]


def test_truncation_error_equals_discarded_tail_single_cut():
    # with all rank lost at one cut the error is the discarded singular-value tail
    L, N = 8, 4
    x = _sector_vector(L, N, 2)
    sv = tt.singular_values(x, L, N, 1)
    y, rho, cb, _, svals = tt.truncate(x, L, N, 0.0, cap=1)
    assert rho[1] == {0: 1, 1: 0} or rho[1] == {0: 0, 1: 1}
    assert cb


def test_truncation_of_exact_low_rank_state_is_identity():
    L, N = 10, 5
    rho = rho_table(L, N, 6)
    x = mps.to_dense(L, N, rho, random_block_mps(L, N, rho, 7))
    y, r2, cb, _, _ = tt.truncate(x, L, N, 0.0, cap=1000)
    assert np.allclose(x, y, atol=1e-12 * np.linalg.norm(x))
    for k in range(1, L):
        for n, c in r2[k].items():
            assert c <= rho[k][n]


def test_cap_bound_and_quasi_optimality():
    L, N = 8, 4
    x = _sector_vector(L, N, 3)
    x /= np.linalg.norm(x)
    y, rho, cb, _, svals = tt.truncate(x, L, N, 0.0, cap=3)
    assert cb
    assert max(sum(r.values()) for r in rho[1:L]) <= 3
    # eq. ttsvdquasiopt, first inequality, with the sequentially computed singular values
    disc = 0.0
    for k in range(1, L):
        sv = svals[k - 1]
        kept = rho[k]
        for n, s in sv.items():
            disc += float(np.sum(s[kept[n]:] ** 2))
    assert np.linalg.norm(x - y) <= math.sqrt(disc) * (1 + 1e-10)


def test_select_rules_ties_cap_and_zeros():
    sv = {0: np.array([3.0, 1.0]), 1: np.array([3.0, 2.0, 1e-14])}
    kept, cb, _ = tt.select(sv, delta=0.0, cap=2)
    assert kept == {0: 1, 1: 1} and cb  # tie at 3.0 -> both, sector order
    kept, cb, _ = tt.select(sv, delta=0.0, cap=100)
    assert kept == {0: 2, 1: 2} and not cb  # 1e-14 is a numerical zero
    kept, cb, _ = tt.select(sv, delta=math.sqrt(1.0 + 1.0) + 1e-9, cap=100)
    assert kept == {0: 1, 1: 2}  # the discarded tail {1.0} fits inside delta^2
    kept, _, _ = tt.select({0: np.array([1e-3])}, delta=1.0, cap=5)
    assert kept == {0: 1}  # never empty


def test_mps_contraction_and_amplitudes():
    L, N = 7, 3
    rho = rho_table(L, N, 5)
    data = random_block_mps(L, N, rho, 11)
    assert mps.size(L, N, rho) == len(data)
    x = mps.to_dense(L, N, rho, data)
    basis = fock.sector_basis(L, N)
    for cfg in basis[::5]:
        assert mps.amplitude(L, N, rho, data, int(cfg)) == pytest.approx(x[cfg], abs=1e-13)
    # particle number: no weight outside the sector
    mask = np.ones(1 << L, bool)
    mask[basis] = False
    assert not np.any(x[mask])


@pytest.mark.parametrize("eps", [1e-1, 1e-3])
def test_parallel_truncation_error_bound_and_ranks(eps):
    L, N = 9, 4
    x = _sector_vector(L, N, 4)
    x /= np.linalg.norm(x)
    y, rho, cb, _ = tt.truncate_parallel(x, L, N, eps, cap=10 ** 6)
    assert not cb
    assert np.linalg.norm(x - y) <= eps * (1 + 1e-12)
    r = tt.ranks(y, L, N)
    for k in range(1, L):
        for n, c in r[k].items():
            assert c <= rho[k][n]


def test_parallel_truncation_of_exact_low_rank_state_is_identity():
    L, N = 10, 5
    rho = rho_table(L, N, 6)
    x = mps.to_dense(L, N, rho, random_block_mps(L, N, rho, 3))
    y, r2, cb, _ = tt.truncate_parallel(x, L, N, 0.0, cap=1000)
    assert np.allclose(x, y, atol=1e-12 * np.linalg.norm(x))


def test_parallel_truncation_single_binding_bond_equals_sequential():
    # when the cap binds at one bond only (and eps = 0), both definitions project once
    L, N = 8, 4
    x = _sector_vector(L, N, 5)
    ranks_full = [sum(v.size for v in tt.singular_values(x, L, N, k).values()) for k in range(1, L)]
    cap = max(ranks_full) - 1
    assert sum(1 for r in ranks_full if r > cap) == 1
    y1, r1, _, _, _ = tt.truncate(x, L, N, 0.0, cap)
    y2, r2, _, _ = tt.truncate_parallel(x, L, N, 0.0, cap)
    assert np.allclose(y1, y2, atol=1e-12)
    assert r1 == r2


@pytest.mark.parametrize("eps", [0.02, 0.1, 0.2])
def test_parallel_truncation_keeps_the_least_ranks_of_the_sqrt_split(eps):
    """Each bond of the simultaneous truncation keeps the least count whose discarded tail
    of x's own singular values is at most eps^2/(L-1) (eq. ttsvdquasiopt read for the
    projectors P_k: x - P_1 Y is an orthogonal sum), and the error obeys
    ||x - y||^2 <= sum of the tails <= eps^2.  A split eps/(L-1) would keep more."""
    L, N = 9, 4
    # a state with decaying singular values: low-rank parts of decreasing weight
    x = sum(w * mps.to_dense(L, N, rho_table(L, N, r), random_block_mps(L, N, rho_table(L, N, r), 20 + r))
            for w, r in ((1.0, 2), (0.3, 4), (0.1, 8))) + 0.02 * _sector_vector(L, N, 7)
    x /= np.linalg.norm(x)
    y, rho, cb, _ = tt.truncate_parallel(x, L, N, eps, cap=10 ** 6)
    assert not cb
    d2 = eps * eps / (L - 1)
    tails = 0.0
    looser = 0
    for k in range(1, L):
        sv = np.sort(np.concatenate([s for s in tt.singular_values(x, L, N, k).values()]))[::-1]
        s = sum(rho[k].values())
        tail = float(np.sum(sv[s:] ** 2))
        assert tail <= d2 * (1 + 1e-12)
        assert float(np.sum(sv[s - 1:] ** 2)) > d2
        tails += tail
        s_lin = int(np.argmax(np.concatenate([np.cumsum((sv ** 2)[::-1])[::-1], [0.0]]) <= (eps / (L - 1)) ** 2))
        looser += s_lin > s
    assert np.linalg.norm(x - y) ** 2 <= tails * (1 + 1e-10) <= eps * eps * (1 + 1e-10)
    assert looser > 0  # the split eps/(L-1) would keep more
