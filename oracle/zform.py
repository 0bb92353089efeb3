"""Algorithm 2 in the paper's own variable x ("z-form"; test infrastructure only).

The iterate is x with A = S H_gamma S and E = S^2, S = sum_k S_k a sum of rank-one diagonal
terms (Section 4.3).  Unlike ``pinvit.run`` (which iterates on psi = S x), every product
with A or E is summed term by term over the pairs (k, k') and the residual is the sorted
sequential sum of its (M^+ - M^- + 1)^2 terms:

1. lambda = sum_{k,k'} <H S_k x, S_k' x> / sum_{k,k'} <S_k x, S_k' x> (eq. exactrq);
   x <- x / ||x||_A.
2. Terms s_{k,k'} = S_k (H_gamma - lambda) S_k' x, exact; eta_res <- min(2 eta_res,
   4/5 zeta_res sum ||s_{k,k'}||) (eq. startetar).
3. res_eta(x): terms sorted by norm (ties: lower k, then lower k'), the leading ones whose
   norms add up to at most eta/3 dropped, then y <- trunc_{eps_j}(y + s_j) with
   eps_j = eta ||s_j|| / (3 sum of the kept norms), finally trunc_{eta/3} (Lemma truncr and
   the recipe after it), so ||res_eta(x) - r(x)|| <= eta.  While ||res_eta|| <
   (1 + 1/zeta) eta (and no cap bound): eta <- 4/5 eta.
4. rho = (1-c)^{-1/2} (||r|| + eta) / ||x||_A (eq. rhobound); stop on the bound of
   eq. everrbound.
5. Ritz step on {x, r/||r||} with the A and E products summed term by term (Rem.
   omegamin), x_* = z_1 x + z_2 r/||r|| with x_*^T E x_* = 1.
6. eta_in = Delta sqrt(lambda_*)/sqrt(1+c) (||x_*||_A = sqrt(lambda_*)); x <- trunc_{eta_in}(x_*),
   the truncation acting on x itself.
"""
from __future__ import annotations

import math

import numpy as np

from . import bounds, fock, precond
from .pinvit import Params, initial_determinant


def a_product(pre, h, v, gamma, a, b):
    """<a, A b> = sum_{k,k'} <S_k a, H_gamma S_k' b>, term by term."""
    d = pre.diagonals()
    hb = [fock.apply_h(h, v, dk * b, gamma) for dk in d]
    return float(sum((dk * a) @ hbk for dk in d for hbk in hb))


def e_product(pre, a, b):
    """<a, E b> = sum_{k,k'} <S_k a, S_k' b>, term by term."""
    d = pre.diagonals()
    return float(sum((dk * a) @ (dk2 * b) for dk in d for dk2 in d))


def residual_terms(pre, h, v, gamma, x, lam):
    """[(||s||, k, k', s)] for s = S_k (H_gamma - lambda) S_k' x, all pairs (k, k')."""
    d = pre.diagonals()
    out = []
    for k2, dk2 in enumerate(d):
        u = dk2 * x
        g = fock.apply_h(h, v, u, gamma) - lam * u
        for k, dk in enumerate(d):
            s = dk * g
            out.append((float(np.linalg.norm(s)), k, k2, s))
    return out


def res_eta(terms, eta, L, N, cap, mode):
    """The sorted sequential truncated sum of the residual terms; returns (r, cap_bound)."""
    order = sorted(terms, key=lambda t: (t[0], t[1], t[2]))
    csum, j0 = 0.0, 0
    for j, t in enumerate(order):
        if csum + t[0] <= eta / 3.0:
            csum += t[0]
            j0 = j + 1
        else:
            break
    rest = order[j0:]
    total = sum(t[0] for t in rest)
    y = np.zeros_like(terms[0][3])
    cap_bound = False
    for t in rest:
        eps_j = eta * t[0] / (3.0 * total) if total > 0 else 0.0
        y, _, cb, _, _ = precond._trunc(y + t[3], L, N, eps_j, cap, mode)
        cap_bound |= cb
    y, _, cb, _, _ = precond._trunc(y, L, N, eta / 3.0, cap, mode)
    return y, cap_bound or cb


def run_z(h, v, N, gamma, prm: Params, x0=None):
    """Algorithm 2 on x; returns (x, history, preconditioner).  History records: lam, E,
    rho, bound, r_norm, eta, retries, cap_bound, terms_dropped, and after a Ritz step
    lam_star and eta_in."""
    L = h.shape[0]
    pre = precond.Preconditioner(h, v, N, gamma, prm.c0, prm.c_lower, prm.c_upper, prm.correction)
    mode = prm.truncation
    eps_num = prm.eps_num if prm.eps_num is not None else 0.5 * (1.0 - prm.c)
    zeta = eps_num / (1.0 + prm.c)
    eta = math.inf
    x = fock.determinant(L, initial_determinant(h, N)) if x0 is None else x0.copy()
    hist = []
    for it in range(prm.max_iter):
        num = a_product(pre, h, v, gamma, x, x)
        den = e_product(pre, x, x)
        lam = num / den
        x = x / math.sqrt(num)
        terms = residual_terms(pre, h, v, gamma, x, lam)
        eta = min(2.0 * eta, 0.8 * zeta * sum(t[0] for t in terms))
        retries = 0
        while True:
            r, cap_bound = res_eta(terms, eta, L, N, prm.cap, mode)
            nr = float(np.linalg.norm(r))
            if nr >= (1.0 + 1.0 / zeta) * eta or cap_bound or retries >= prm.max_retries:
                break
            eta *= 0.8
            retries += 1
        rho = (nr + eta) / math.sqrt(1.0 - prm.c)
        bound = bounds.eigvec_error_bound(rho, prm.delta)
        rec = dict(it=it, lam=lam, E=lam - gamma, rho=rho, bound=bound, r_norm=nr, eta=eta,
                   retries=retries, cap_bound=bool(cap_bound))
        if bound <= prm.tau:
            rec["stop"] = True
            hist.append(rec)
            break
        rh = r / nr
        hm = np.array([[1.0, a_product(pre, h, v, gamma, x, rh)],
                       [0.0, a_product(pre, h, v, gamma, rh, rh)]])
        hm[1, 0] = hm[0, 1]
        e01 = e_product(pre, x, rh)
        mm = np.array([[e_product(pre, x, x), e01], [e01, e_product(pre, rh, rh)]])
        lam_s, z = bounds.ritz2(hm, mm)
        q = math.sqrt(lam_s / (lam_s + prm.t_eig * (lam - lam_s)))
        eta_in = bounds.delta_a(rho, q) * math.sqrt(lam_s) / math.sqrt(1.0 + prm.c)
        x, _, cb, _, _ = precond._trunc(z[0] * x + z[1] * rh, L, N, eta_in, prm.cap, mode)
        rec.update(lam_star=lam_s, eta_in=eta_in, cap_bound_update=bool(cb))
        hist.append(rec)
    return x, hist, pre
