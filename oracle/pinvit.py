"""Algorithm 2 (perturbed inverse inner iteration) in the physical variable (oracle).

The paper iterates on x with A = S H_gamma S, E = S^2 (Section 3.1, eqs. Hevpprecond,
basicpinvit).  With psi = S x one has lambda(x) = <H_gamma psi, psi>/<psi, psi>,
the preconditioned residual S r(x) = S^2 (H_gamma - lambda) psi, ||x||_A^2 =
<H_gamma psi, psi>, and the Ritz space span{x, res} maps to span{psi, S res}.  This
module runs Alg. 2 on psi; truncations act on psi (a reading, listed in the design doc).

One iteration (every step on full vectors, truncations by ``tt.truncate``):

1. psi <- psi/||psi||; lambda = <psi, H_gamma psi> exactly (eq. exactrq).
2. eta_res <- min(2 eta_res, 4/5 zeta_res est), zeta_res = eps_num/(1+c) (Lemma truncr,
   eq. startetar); est = s_max ||trunc_{0,cap}(trunc_{0,cap}(H psi) - lambda psi)|| at the
   first iteration, afterwards ||s|| of the previous iteration times its last decrease
   ratio (capped at 1).
3. y = trunc_{e1}(H_gamma psi); r = trunc_{e2}(y - lambda psi); s = S_sorted(r; e3) with
   e1 = e2 = eta/(3 s_max), e3 = eta/3, so ||s - S(H_gamma - lambda)psi|| <= eta.
4. while ||s|| < (1 + 1/zeta) eta and no cap bound: eta <- 4/5 eta, redo 3 (Section 5.3.1).
5. rho^n = (1-c)^{-1/2} (||s|| + eta)/||x||_A (eq. rhobound); stop when the bound of
   eq. everrbound is <= tau.
6. p = S_sorted(s; s_max eta/3); 2x2 Ritz problem on {psi, p/||p||} (Rem. omegamin).
   If p vanishes (the residual fell below the truncation tolerances, as happens on a
   sector of dimension 2), psi is an eigenvector to those tolerances and the run stops.
7. eta_in = Delta ||x_*||_A/sqrt(1+c) with Delta from sqrt(1-Delta^2) - rho Delta =
   sqrt(lam_*/(lam_* + t_eig (lambda - lam_*))) (Lemma on iterate truncation);
   psi <- trunc_{s_min eta_in}(v_1 psi + v_2 p/||p||).

``run_outer`` is Algorithm 3 (outer iteration, Section 5.6 / Thm. quasioptr) on top of it.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import bounds, fock, precond, tt


@dataclasses.dataclass
class Params:
    cap: int = 16
    max_iter: int = 20
    tau: float = 1e-10
    c: float = 0.5
    delta: float = 10.0
    c0: float = 0.1
    c_lower: float = 1.0
    c_upper: float = 1.0
    t_eig: float = 0.5
    eps_num: float | None = None
    max_retries: int = 30
    truncation: str = "sequential"  # or "parallel" (tt.truncate_parallel)
    correction: object = None  # L x (N+1) learned correction of theta (oracle.learned)


def initial_determinant(h: np.ndarray, N: int):
    """Orbitals of the starting determinant: the N smallest h_ii, ties to the lower index
    (Section 7.1.4: the lowest-energy unit vector e_1)."""
    return sorted(np.argsort(np.diag(h), kind="stable")[:N].tolist())


def run(h, v, N, gamma, prm: Params, psi0=None):
    L = h.shape[0]
    pre = precond.Preconditioner(h, v, N, gamma, prm.c0, prm.c_lower, prm.c_upper, prm.correction)
    mode = prm.truncation

    def trunc(x, eps):
        return precond._trunc(x, L, N, eps, prm.cap, mode)
    eps_num = prm.eps_num if prm.eps_num is not None else 0.5 * (1.0 - prm.c)
    zeta = eps_num / (1.0 + prm.c)
    eta = math.inf
    psi = fock.determinant(L, initial_determinant(h, N)) if psi0 is None else psi0.copy()
    hist = []
    s_prev = s_prev2 = None
    for it in range(prm.max_iter):
        psi = psi / np.linalg.norm(psi)
        hpsi = fock.apply_h(h, v, psi, gamma)
        lam = float(psi @ hpsi)
        if s_prev is None:
            y0 = trunc(hpsi, 0.0)[0]
            r0 = trunc(y0 - lam * psi, 0.0)[0]
            est = pre.s_max * float(np.linalg.norm(r0))
        elif s_prev2 is None or s_prev2 <= 0.0:
            est = s_prev
        else:
            est = s_prev * min(1.0, s_prev / s_prev2)
        eta = min(2.0 * eta, 0.8 * zeta * est)
        retries = 0
        margin = math.inf
        while True:
            e12 = eta / (3.0 * pre.s_max)
            y, _, cb1, m1, _ = trunc(hpsi, e12)
            r, rho_r, cb2, m2, _ = trunc(y - lam * psi, e12)
            s, cb3, _, m3 = precond.apply_sorted(pre, r, eta / 3.0, prm.cap, N, mode)
            cap_bound = cb1 or cb2 or cb3
            ns = float(np.linalg.norm(s))
            mret = min(m1, m2, m3)
            if ns >= (1.0 + 1.0 / zeta) * eta or cap_bound or retries >= prm.max_retries:
                margin = min(margin, mret)
                break
            eta *= 0.8
            retries += 1
        p, cb4, _, m4 = precond.apply_sorted(pre, s, pre.s_max * eta / 3.0, prm.cap, N, mode)
        nr = float(np.linalg.norm(r))
        rho = (ns + eta) / (math.sqrt(1.0 - prm.c) * math.sqrt(lam))
        bound = bounds.eigvec_error_bound(rho, prm.delta)
        rec = dict(it=it, lam=lam, E=lam - gamma, rho=rho, bound=bound, r_norm=nr,
                   s_norm=ns, eta=eta, retries=retries, cap_bound=bool(cap_bound or cb4),
                   margin=min(margin, m4))
        if bound <= prm.tau:
            rec["stop"] = True
            hist.append(rec)
            break
        npn = float(np.linalg.norm(p))
        if npn == 0.0:
            # the direction vanished under the truncation tolerances: psi is an eigenvector
            # to those tolerances and the iteration stops (a reading for this degenerate case)
            rec["stop"] = True
            rec["direction_vanished"] = True
            hist.append(rec)
            break
        z2 = p / npn
        hz2 = fock.apply_h(h, v, z2, gamma)
        o12 = float(psi @ z2)
        hm = np.array([[lam, float(psi @ hz2)], [float(psi @ hz2), float(z2 @ hz2)]])
        mm = np.array([[1.0, o12], [o12, 1.0]])
        lam_s, vv = bounds.ritz2(hm, mm)
        q = math.sqrt(lam_s / (lam_s + prm.t_eig * (lam - lam_s)))
        da = bounds.delta_a(rho, q)
        eta_in = da * math.sqrt(lam_s) / math.sqrt(1.0 + prm.c)
        eta_psi = eta_in * pre.s_min
        psi, rho_tab, cb5, m5, _ = trunc(vv[0] * psi + vv[1] * z2, eta_psi)
        rec.update(lam_star=lam_s, v=vv.copy(), eta_psi=eta_psi, rho_tab=rho_tab,
                   cap_bound_update=bool(cb5), margin=min(rec["margin"], m5))
        hist.append(rec)
        s_prev2, s_prev = s_prev, ns
    return psi, hist, pre


def outer_constants(L: int, c: float, alpha: float):
    """kappa of eq. kappadef, theta and eta_0 of Algorithm 3 (D = 1)."""
    kappa = math.sqrt((1.0 + c) / (1.0 - c)) * math.sqrt(L - 1)
    ak = (1.0 + alpha) * kappa
    theta = ak / (2.0 * (1.0 + ak))
    return kappa, theta, 1.0 / (2.0 * theta)


def run_outer(h, v, N, gamma, prm: Params, alpha: float = 1.0, tol: float = 1e-8, max_outer: int = 20):
    """Algorithm 3: for m = 0, 1, ...: y+ = PINVIT(y^m) run until the eigenvector bound of
    eq. everrbound is below tau_m = eta^m / (2 (1 + (1+alpha) kappa)); stop when the
    relative eigenvalue bound of eq. releigerr of its last residual bound rho is below tol;
    otherwise y^{m+1} = trunc_{theta eta^m}(y+) and eta^{m+1} = eta^m / 2.  Iterates are
    normalised; the truncation tolerance is converted to psi = S x with s_min, as for the
    inner iterate truncation (a reading)."""
    L = h.shape[0]
    kappa, theta, eta = outer_constants(L, prm.c, alpha)
    ak = (1.0 + alpha) * kappa
    psi = None
    outer = []
    for m in range(max_outer):
        tau_m = eta / (2.0 * (1.0 + ak))
        inner = dataclasses.replace(prm, tau=tau_m)
        y, hist, pre = run(h, v, N, gamma, inner, psi0=psi)
        last = hist[-1]
        rel = bounds.rel_eig_bound(last["rho"], prm.delta)
        rec = dict(m=m, eta=eta, tau=tau_m, inner=len(hist), lam=last["lam"], E=last["E"],
                   rho=last["rho"], rel_bound=rel, converged_inner=bool(last.get("stop")))
        y = y / np.linalg.norm(y)
        if rel < tol:
            rec["stop"] = True
            outer.append(rec)
            return y, outer
        eps = pre.s_min * theta * eta
        psi, rho_tab, cb, margin, _ = precond._trunc(y, L, N, eps, prm.cap, prm.truncation)
        rec.update(trunc_eps=eps, rho_tab=rho_tab, cap_bound=bool(cb), margin=margin,
                   trunc_err=float(np.linalg.norm(psi - y)))
        outer.append(rec)
        eta *= 0.5
    return psi, outer
