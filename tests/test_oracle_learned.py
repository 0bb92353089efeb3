"""Pins of the oracle's learned preconditioner correction (an extension, not in the paper):
the exact diagonal against the dense Hamiltonian, the corrected t_min/t_max against
enumeration, the corrected S against its definition on every determinant, the zero
correction against the plain S, the bfloat16 rounding against its bit definition, the
gradient against finite differences, and training lowering the misfit."""
import itertools
import math

import numpy as np
import pytest

from oracle import fock, learned, pinvit, precond
from synth import init_params, make_problem, sample_determinants


@pytest.fixture(scope="module")
def small():
    return make_problem("dense", 6, 3, 3)


def _features(p, N, x=None, lam=None):
    th = precond.theta(p.h, p.v, N, p.gamma)
    L = len(th)
    if x is None:
        x = fock.determinant(L, pinvit.initial_determinant(p.h, N))
    if lam is None:
        lam = float(x @ fock.apply_h(p.h, p.v, x, p.gamma)) / float(x @ x)
    return th, learned.features(th, np.diag(p.h), learned.densities(x), lam, N)


def test_exact_diagonal_is_the_dense_diagonal(small):
    p, L, N = small, 6, 3
    masks = fock.sector_basis(L, N)
    want = [fock.apply_h(p.h, p.v, np.eye(1 << L)[m], p.gamma)[m] for m in masks]
    got = learned.exact_diagonal(p.h, p.v, p.gamma, masks)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def test_bf16_rounding_matches_the_bit_definition():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, 1.0 + 2 ** -8 + 2 ** -20, -3.14159, 0.0],
                 dtype=np.float32)
    # halfway cases go to the even neighbour; above halfway rounds up
    want = [1.0, 1.0, 1.0 + 4 * 2 ** -8, 1.0, 1.0 + 2 ** -7, -3.140625, 0.0]
    assert list(learned.bf16(x)) == want


def test_corrected_range_and_terms_by_enumeration(small):
    p, L, N = small, 6, 3
    th, X = _features(p, N)
    rng = np.random.default_rng(1)
    delta = 0.3 * learned.delta_max(th) * rng.uniform(-1, 1, size=(L, N + 1))
    sums = {}
    for occ in itertools.combinations(range(L), N):
        sums[sum(1 << i for i in occ)] = sum(th[i] + delta[i, k] for k, i in enumerate(occ))
    lo, hi = learned.t_range(th, delta, N)
    assert lo == pytest.approx(min(sums.values()), rel=1e-14)
    assert hi == pytest.approx(max(sums.values()), rel=1e-14)
    pre = precond.Preconditioner(p.h, p.v, N, p.gamma, delta=delta)
    assert pre.t_min == pytest.approx(lo, rel=1e-14)
    d = pre.diagonals()
    for m, dm in enumerate(d):
        for mask, s in sums.items():
            assert dm[mask] == pytest.approx(pre.alpha[m] * math.exp(-pre.beta[m] * s), rel=1e-12)
    # S stays within [s_min, s_max] on the sector (S(t) decreases in t)
    tot = sum(d)
    vals = [tot[mk] for mk in sums]
    assert min(vals) >= pre.s_min * (1 - 1e-12) and max(vals) <= pre.s_max * (1 + 1e-12)


def test_zero_correction_is_the_plain_preconditioner(small):
    p, L, N = small, 6, 3
    a = precond.Preconditioner(p.h, p.v, N, p.gamma)
    b = precond.Preconditioner(p.h, p.v, N, p.gamma, delta=np.zeros((L, N + 1)))
    # equal up to the order of the sums (sorted theta against the path recursion)
    np.testing.assert_allclose([b.t_min, b.t_max, b.s_min, b.s_max], [a.t_min, a.t_max, a.s_min, a.s_max], rtol=1e-14)
    assert a.M == b.M
    for x, y in zip(a.diagonals(), b.diagonals()):
        np.testing.assert_allclose(x, y, rtol=1e-13)


def test_correction_is_bounded(small):
    p, N = small, 3
    th, X = _features(p, N)
    w = init_params(0, out_scale=50.0)  # a saturated output
    dm = learned.delta_max(th)
    c = learned.correction(w, X, dm, 6, N)
    assert np.all(np.abs(c) <= dm) and np.all(th[:, None] + c > 0)


def test_gradient_matches_finite_differences(small):
    p, L, N = small, 6, 3
    th, X = _features(p, N)
    masks = sample_determinants(L, N, 40, seed=2)
    tg = learned.exact_diagonal(p.h, p.v, p.gamma, masks)
    dm = learned.delta_max(th)
    # parameters already on the bfloat16 grid, perturbed by exactly representable steps
    w = learned.bf16(init_params(3, out_scale=1.0))
    loss, g = learned.loss_grad(w, X, dm, th, masks, tg, N)
    rng = np.random.default_rng(4)
    for k in rng.choice(len(w), size=12, replace=False):
        hstep = 2.0 ** (math.floor(math.log2(abs(w[k]) + 1e-30)) - 3) if w[k] != 0 else 2.0 ** -12
        wp, wm = w.copy(), w.copy()
        wp[k] += hstep
        wm[k] -= hstep
        fd = (learned.loss_grad(wp, X, dm, th, masks, tg, N)[0] - learned.loss_grad(wm, X, dm, th, masks, tg, N)[0]) / (2 * hstep)
        assert fd == pytest.approx(g[k], rel=2e-2, abs=1e-6 * np.abs(g).max())


def test_training_lowers_the_misfit(small):
    p, L, N = small, 6, 3
    th, X = _features(p, N)
    masks = sample_determinants(L, N, 64, seed=5)
    tg = learned.exact_diagonal(p.h, p.v, p.gamma, masks)
    dm = learned.delta_max(th)
    w, losses = learned.train(init_params(0), X, dm, th, masks, tg, N, steps=30, lr=1e-3)
    assert w.dtype == np.float32
    assert losses[-1] < 0.8 * losses[0]


def test_corrected_run_reaches_the_same_eigenvalue(small):
    # a preconditioner changes the path, not the fixed point: Algorithm 2 with a trained
    # correction ends at the lowest eigenvalue of exact diagonalisation
    p, L, N = small, 6, 3
    th, X = _features(p, N)
    masks = sample_determinants(L, N, 64, seed=5)
    tg = learned.exact_diagonal(p.h, p.v, p.gamma, masks)
    w, _ = learned.train(init_params(0), X, learned.delta_max(th), th, masks, tg, N, steps=20, lr=1e-3)
    corr = learned.correction(w, X, learned.delta_max(th), L, N)
    assert np.abs(corr).max() > 0
    ed = fock.lowest_eigs(p.h, p.v, N, p.gamma, k=1)[0]
    prm = pinvit.Params(cap=64, max_iter=40, tau=1e-9, correction=corr)
    _, hist, _ = pinvit.run(p.h, p.v, N, p.gamma, prm)
    assert 0 <= hist[-1]["lam"] - ed <= 1e-7 * abs(ed)


def _solve_samples(p, L, N, seed):
    """A residual of the method (first iterate of Algorithm 2) and its exact solve on all
    determinants of the sector."""
    x = fock.determinant(L, pinvit.initial_determinant(p.h, N))
    hx = fock.apply_h(p.h, p.v, x, p.gamma)
    r = hx - float(x @ hx) * x
    t = learned.exact_solve(p.h, p.v, N, p.gamma, r)
    masks = [int(m) for m in fock.sector_basis(L, N)]
    return r, t, masks


def test_exact_solve_inverts_the_sector_hamiltonian(small):
    p, L, N = small, 6, 3
    r, t, masks = _solve_samples(p, L, N, 0)
    assert np.abs(fock.apply_h(p.h, p.v, t, p.gamma) - r).max() <= 1e-12 * np.abs(r).max()
    # nothing outside the sector
    other = np.setdiff1d(np.arange(1 << L), fock.sector_basis(L, N))
    assert np.all(t[other] == 0.0)


def test_solve_gradient_matches_finite_differences(small):
    p, L, N = small, 6, 3
    th, X = _features(p, N)
    r, t, masks = _solve_samples(p, L, N, 0)
    dm = learned.delta_max(th)
    w = learned.bf16(init_params(3, out_scale=1.0))
    loss, g = learned.solve_loss_grad(w, X, dm, th, masks, r[masks], t[masks], N)
    # the loss at a zero correction is the misfit of the plain diagonal, a number in (0, 1]
    w0 = np.zeros_like(w)
    l0, _ = learned.solve_loss_grad(w0, X, dm, th, masks, r[masks], t[masks], N)
    d0 = learned.approx_diagonal(th, np.zeros((L, N + 1)), masks)
    tv = t[masks]
    assert l0 == pytest.approx(np.sum((r[masks] / d0 - tv) ** 2) / np.sum(tv * tv), rel=1e-12)
    rng = np.random.default_rng(6)
    for k in rng.choice(len(w), size=12, replace=False):
        # steps of two bfloat16 units: the misfit is far from quadratic in the parameters
        hstep = 2.0 ** (math.floor(math.log2(abs(w[k]) + 1e-30)) - 6) if w[k] != 0 else 2.0 ** -14
        wp, wm = w.copy(), w.copy()
        wp[k] += hstep
        wm[k] -= hstep
        fp = learned.solve_loss_grad(wp, X, dm, th, masks, r[masks], tv, N)[0]
        fm = learned.solve_loss_grad(wm, X, dm, th, masks, r[masks], tv, N)[0]
        assert (fp - fm) / (2 * hstep) == pytest.approx(g[k], rel=2e-2, abs=1e-6 * np.abs(g).max())
