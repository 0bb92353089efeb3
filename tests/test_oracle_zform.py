"""Pins of the oracle's z-form Algorithm 2 (products with A and E summed term by term, the
residual as the sorted sum of its M^2 terms): equivalence with the psi-form when nothing is
truncated (the reading that the build iterates on psi = S x), the error bound of the sorted
residual sum against the exact residual, and the variational bound."""
import math

import numpy as np
import pytest

from oracle import fock, pinvit, zform
from synth import make_problem


@pytest.fixture(scope="module")
def l8():
    return make_problem("decayed", 8, 4, 0)


def test_zform_equals_psi_form_without_truncation(l8):
    # eps_num and t_eig near zero make every truncation tolerance negligible; then the
    # Ritz spaces {x, res(x)} and {S x, S^2 (H - lambda) S x} coincide and so do the energies
    p = l8
    prm = pinvit.Params(cap=64, max_iter=10, tau=1e-12, eps_num=1e-13, t_eig=1e-13)
    _, hz, _ = zform.run_z(p.h, p.v, 4, p.gamma, prm)
    _, hp, _ = pinvit.run(p.h, p.v, 4, p.gamma, prm)
    assert len(hz) == len(hp) == 10
    for a, b in zip(hz, hp):
        assert abs(a["E"] - b["E"]) <= 1e-12 * abs(b["E"])


def test_sorted_residual_sum_meets_its_tolerance(l8):
    p = l8
    pre = pinvit.precond.Preconditioner(p.h, p.v, 4, p.gamma)
    rng = np.random.default_rng(5)
    basis = fock.sector_basis(8, 4)
    x = np.zeros(1 << 8)
    x[basis] = rng.standard_normal(len(basis))
    lam = zform.a_product(pre, p.h, p.v, p.gamma, x, x) / zform.e_product(pre, x, x)
    # the exact residual through the dense S (one product, not the term sum)
    sx = pre.apply_exact(x)
    r = pre.apply_exact(fock.apply_h(p.h, p.v, sx, p.gamma) - lam * sx)
    terms = zform.residual_terms(pre, p.h, p.v, p.gamma, x, lam)
    for eta_rel in (1e-1, 1e-3, 1e-6):
        eta = eta_rel * np.linalg.norm(r)
        got, cb = zform.res_eta(terms, eta, 8, 4, 10 ** 6, "sequential")
        assert not cb
        assert np.linalg.norm(got - r) <= eta * (1 + 1e-10)
    # the Rayleigh quotient of eq. exactrq through the dense S
    assert lam == pytest.approx(float(sx @ fock.apply_h(p.h, p.v, sx, p.gamma)) / float(sx @ sx), rel=1e-13)


def test_zform_energies_are_variational_and_converge(l8):
    p = l8
    ed = fock.lowest_eigs(p.h, p.v, 4, p.gamma, 1)[0]
    prm = pinvit.Params(cap=16, max_iter=20, tau=1e-12)
    _, hz, _ = zform.run_z(p.h, p.v, 4, p.gamma, prm)
    for rec in hz:
        assert rec["lam"] >= ed - 1e-12 * abs(ed)
        if "lam_star" in rec:
            assert rec["lam_star"] <= rec["lam"] * (1 + 1e-13)
    assert hz[-1]["lam"] - ed <= 1e-4 * abs(ed)
    assert hz[-1]["lam"] < hz[1]["lam"]
