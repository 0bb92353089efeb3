"""Pins of the oracle's Algorithm 4 (subspace iteration, Section 6): against exact
diagonalisation of the N-particle sector, the min-max property of Ritz values, the
one-column case (Algorithm 2), and the starting determinants."""
import math

import numpy as np
import pytest

from oracle import fock, pinvit, precond, subspace
from synth import make_problem


@pytest.fixture(scope="module")
def l8():
    p = make_problem("decayed", 8, 4, 0)
    ed = fock.lowest_eigs(p.h, p.v, 4, p.gamma, 4)
    prm = pinvit.Params(cap=64, max_iter=36, tau=1e-12)
    X, hist, _ = subspace.run_subspace(p.h, p.v, 4, p.gamma, prm, 3)
    return p, ed, X, hist


def test_subspace_reaches_the_lowest_eigenvalues(l8):
    p, ed, X, hist = l8
    lam = hist[-1]["lam"]
    # the lowest two converge fast; the third more slowly (its gap to the fourth is smaller)
    assert abs(lam[0] - ed[0]) <= 1e-10 * abs(ed[0])
    assert abs(lam[1] - ed[1]) <= 1e-8 * abs(ed[1])
    assert abs(lam[2] - ed[2]) <= 1e-3 * abs(ed[2])


def test_ritz_values_bound_the_eigenvalues_from_above(l8):
    # min-max: the i-th Ritz value of any D-dimensional subspace is >= the i-th eigenvalue
    p, ed, X, hist = l8
    for rec in hist:
        lam = rec["lam"]
        assert np.all(np.diff(lam) >= 0)
        assert np.all(lam >= ed[:3] - 1e-11 * np.abs(ed[:3]))
        if "lam_star" in rec:
            assert np.all(rec["lam_star"] >= ed[:3] - 1e-11 * np.abs(ed[:3]))
            # the 2D-dimensional Ritz space contains span Psi: its values are not larger
            assert np.all(rec["lam_star"] <= lam + 1e-11 * np.abs(lam))


def test_one_column_is_algorithm_2():
    p = make_problem("decayed", 8, 4, 1)
    prm = pinvit.Params(cap=64, max_iter=8, tau=1e-12)
    _, h1, _ = subspace.run_subspace(p.h, p.v, 4, p.gamma, prm, 1)
    _, h2, _ = pinvit.run(p.h, p.v, 4, p.gamma, prm)
    assert len(h1) == len(h2)
    for a, b in zip(h1, h2):
        assert abs(a["E"][0] - b["E"]) <= 1e-12 * abs(b["E"])
        assert abs(a["rho"][0] - b["rho"]) <= 1e-9 * b["rho"]


def test_start_determinants_are_the_lowest_single_excitations():
    h = np.diag([0.0, 1.0, 2.5, 3.0, 3.2, 9.0])
    dets = subspace.start_determinants(h, 3, 4)
    assert dets[0] == [0, 1, 2]
    # excitations i -> a ordered by h_aa - h_ii: 2->3 (0.5), 2->4 (0.7), 1->3 (2.0)
    assert dets[1:] == [[0, 1, 3], [0, 1, 4], [0, 2, 3]]
    for d in dets:
        assert len(set(d)) == 3


def test_rank_cap_keeps_ritz_values_above_the_eigenvalues():
    # with a binding rank cap the iterates are truncated, the min-max bound still holds
    p = make_problem("decayed", 8, 4, 2)
    ed = fock.lowest_eigs(p.h, p.v, 4, p.gamma, 2)
    prm = pinvit.Params(cap=4, max_iter=10, tau=1e-12)
    _, hist, _ = subspace.run_subspace(p.h, p.v, 4, p.gamma, prm, 2)
    for rec in hist:
        assert np.all(rec["lam"] >= ed - 1e-11 * np.abs(ed))


def test_sector_of_dimension_2d_is_solved_in_one_step():
    # with 2D equal to the sector dimension the Ritz basis of the first step spans the
    # sector: its Ritz values are the D lowest eigenvalues, and the next directions vanish
    for L, N, D in [(4, 1, 2), (4, 2, 3), (6, 5, 3)]:
        p = make_problem("dense", L, N, 3)
        assert 2 * D == math.comb(L, N)
        w = fock.lowest_eigs(p.h, p.v, N, p.gamma, k=D)
        prm = pinvit.Params(cap=8, max_iter=8, tau=1e-12, c=0.5, delta=10.0)
        _, hist, _ = subspace.run_subspace(p.h, p.v, N, p.gamma, prm, D)
        assert len(hist) == 2 and hist[-1]["stop"] and hist[-1]["direction_vanished"]
        assert np.allclose(hist[0]["lam_star"], w, rtol=1e-12, atol=0)
        assert np.allclose(hist[-1]["lam"], w, rtol=1e-12, atol=0)


def test_sector_below_2d_is_rejected():
    p = make_problem("dense", 3, 1, 3)
    with pytest.raises(ValueError):
        subspace.run_subspace(p.h, p.v, 1, p.gamma, pinvit.Params(cap=8, max_iter=2), 2)


# ---- joint representation (Section 6.2)

def _sector_columns(L, N, D, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((1 << L, D))
    X[[bin(i).count("1") != N for i in range(1 << L)]] = 0.0
    return X


@pytest.mark.parametrize("mode", ["sequential", "parallel"])
def test_joint_truncation_of_one_column_is_the_plain_truncation(mode):
    from oracle import tt
    L, N = 8, 4
    X = _sector_columns(L, N, 1, 3)
    for eps, cap in ((0.3, 1000), (0.0, 5), (1.0, 7)):
        if mode == "sequential":
            Y, rho, cb, _ = tt.truncate_joint(X, L, N, eps, cap)
            y, rho1, cb1, _, _ = tt.truncate(X[:, 0], L, N, eps, cap)
        else:
            Y, rho, cb, _ = tt.truncate_parallel_joint(X, L, N, eps, cap)
            y, rho1, cb1, _ = tt.truncate_parallel(X[:, 0], L, N, eps, cap)
        assert np.abs(Y[:, 0] - y).max() <= 1e-12 and cb == cb1
        assert all(rho[k] == rho1[k] for k in range(1, L))


@pytest.mark.parametrize("eps", [0.5, 2.0, 5.0])
def test_joint_truncation_error_and_shared_ranks(eps):
    """||X - Y||_F <= eps over all columns together, and every column of Y has the joint
    ranks (the column index sits after orbital L)."""
    from oracle import tt
    L, N, D = 9, 4, 3
    # columns with decaying singular values: shared low-rank part plus small noise
    base = _sector_columns(L, N, 1, 5)[:, 0]
    X = np.stack([base * (1 + 0.1 * j) for j in range(D)], axis=1) + 0.05 * _sector_columns(L, N, D, 6)
    for fn in (tt.truncate_joint, tt.truncate_parallel_joint):
        Y, rho, cb, _ = fn(X, L, N, eps, 10 ** 6)
        assert not cb
        assert np.linalg.norm(X - Y) <= eps * (1 + 1e-12)
        for k in range(1, L):
            for n, (_, _, B) in tt.joint_blocks(Y, L, N, k).items():
                s = np.linalg.svd(B, compute_uv=False) if B.size else np.zeros(0)
                assert np.sum(s > 1e-10 * max(s.max(initial=0), 1e-300)) <= rho[k][n]


def test_joint_sorted_sum_of_one_column_is_the_plain_one():
    L, N = 8, 4
    p = make_problem("dense", L, N, 0)
    pre = precond.Preconditioner(p.h, p.v, N, p.gamma)
    X = _sector_columns(L, N, 1, 7)
    for eta in (1e-3, 0.3):
        Y, cb = precond.apply_sorted_joint(pre, X, eta, 1000, N)
        y, cb1, _, _ = precond.apply_sorted(pre, X[:, 0], eta, 1000, N)
        assert np.abs(Y[:, 0] - y).max() <= 1e-13 and cb == cb1


def test_joint_subspace_iteration_one_column_is_the_separate_one():
    p = make_problem("dense", 8, 4, 0)
    prm = pinvit.Params(cap=16, max_iter=10, tau=0.0, c=0.5, delta=10.0)
    _, hj, _ = subspace.run_subspace_joint(p.h, p.v, 4, p.gamma, prm, 1)
    _, hs, _ = subspace.run_subspace(p.h, p.v, 4, p.gamma, prm, 1)
    assert len(hj) == len(hs)
    for a, b in zip(hj, hs):
        assert abs(a["E"][0] - b["E"][0]) <= 1e-12 * abs(b["E"][0])


@pytest.mark.parametrize("D", [2, 3])
def test_joint_subspace_iteration_reaches_the_lowest_eigenvalues(D):
    """With a cap that holds the columns' summed ranks the joint iteration converges to the
    D lowest eigenvalues of exact diagonalisation, every Ritz value staying above its
    eigenvalue (min-max)."""
    L, N = 8, 4
    p = make_problem("dense", L, N, 0)
    w = fock.lowest_eigs(p.h, p.v, N, p.gamma, k=D + 1)
    prm = pinvit.Params(cap=64, max_iter=60, tau=1e-8, c=0.5, delta=w[D] / (w[D] - w[0]))
    _, hist, _ = subspace.run_subspace_joint(p.h, p.v, N, p.gamma, prm, D)
    for r in hist:
        assert np.all(r["lam"] >= w[:D] - 1e-10)
        if "lam_star" in r:
            assert np.all(r["lam_star"] <= r["lam"] + 1e-10)
    assert abs(hist[-1]["lam"][0] - w[0]) <= 1e-8 * w[0]
    assert np.all(np.abs(hist[-1]["lam"] - w[:D]) <= 1e-2 * w[:D])
