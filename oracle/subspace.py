"""Algorithm 4 (perturbed inverse inner subspace iteration, Section 6) in the physical
variable psi = S x (oracle; test infrastructure only).

The D columns X = (x_1, ..., x_D) are kept as D separate vectors.  The paper stores them
as one joint block MPS whose extra core carries the column index (Section 6.2), so that
X <- X V costs nothing and one truncation acts on all columns together.  Here the
normalisation X <- X V is done exactly on the full vectors, and every truncation of the
iterate acts on each column with the whole tolerance, the worst case that the paper
assumes for the joint truncation (all of the error in one column).

With psi_i = S x_i the generalised products become X^T A Y = Psi^T H_gamma Phi and
X^T E Y = Psi^T Phi (A = S H_gamma S, E = S^2), as in the one-vector case.

One iteration:

1. Rayleigh-Ritz on span Psi: Psi^T H Psi V = Psi^T Psi V Lambda with V^T Psi^T Psi V = I,
   eigenvalues ascending; Psi <- Psi V (E-orthonormal columns, Lambda = diag(lambda_i)).
2. eta_res <- min(2 eta_res, 4/5 zeta_res est) (eq. startetar); est = s_max times the
   largest column norm of trunc_0(trunc_0(H psi_i) - lambda_i psi_i) at the first
   iteration, afterwards the largest ||s_i|| of the previous iteration times its last
   decrease ratio (capped at 1), as for D = 1.
3. Per column: y_i = trunc_{e1}(H psi_i); r_i = trunc_{e2}(y_i - lambda_i psi_i);
   s_i = S_sorted(r_i; e3), e1 = e2 = eta/(3 s_max), e3 = eta/3.
4. While min_i ||s_i|| < (1 + 1/zeta) eta (and no cap bound): eta <- 4/5 eta, redo 3.
5. rho_i = (1-c)^{-1/2} (||s_i|| + eta)/||x_i||_A; the eigenvector bound of the first
   column decides termination (eq. everrbound).
6. p_i = S_sorted(s_i; s_max eta/3); if every p_i vanished under the truncation
   tolerances the columns span an invariant subspace to those tolerances and the
   iteration stops (a reading for this degenerate case; a run where only some vanish is
   rejected).  Rayleigh-Ritz on the 2D vectors
   (psi_1..psi_D, p_1/||p_1||..p_D/||p_D||): B W = M W Lambda_*, lowest D eigenvalues,
   W^T M W = I (the rescaling by the norms of eq. subspacerescale is the normalisation of
   the p_i; the psi_i are E-normalised already).
7. eta_in = (1+c)^{-1/2} min_i ||x_*i||_A Delta_i with
   sqrt(1-Delta_i^2) - rho_i Delta_i = sqrt(lambda_*i/(lambda_*i + t_eig(lambda_i -
   lambda_*i))); each new column psi_i <- trunc_{s_min eta_in}(sum_j W_ji b_j).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import bounds, fock, precond
from .pinvit import Params, initial_determinant


def start_determinants(h: np.ndarray, N: int, D: int):
    """D starting determinants: the lowest one of Alg. 2 (N smallest h_ii) and the single
    excitations i -> a from it with the smallest h_aa - h_ii (ties: lower i, then lower a).
    A reading: the paper takes the first D unit vectors of its ordered basis."""
    L = h.shape[0]
    occ = initial_determinant(h, N)
    virt = [a for a in range(L) if a not in occ]
    ex = sorted(((h[a, a] - h[i, i], i, a) for i in occ for a in virt), key=lambda t: (t[0], t[1], t[2]))
    out = [occ]
    for _, i, a in ex[:max(D - 1, 0)]:
        out.append(sorted([o for o in occ if o != i] + [a]))
    if len(out) < D:
        raise ValueError("not enough single excitations for D starting vectors")
    return out


def _gen_eig_lowest(B: np.ndarray, M: np.ndarray, k: int):
    """Lowest k eigenpairs of the symmetric pencil (B, M), M positive definite, eigenvectors
    M-orthonormal; the largest-magnitude entry of each vector is made positive."""
    w, V = scipy.linalg.eigh(B, M)
    w, V = w[:k], V[:, :k].copy()
    for j in range(k):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return w, V


def run_subspace(h, v, N, gamma, prm: Params, D: int, X0=None):
    """Algorithm 4 on D columns; returns (Psi as an n x D array, history, preconditioner).
    Each history record holds lam (the D Rayleigh quotients), E = lam - gamma, rho (D
    residual bounds), bound (first column), eta, retries, and after a Ritz step lam_star
    and eta_psi."""
    L = h.shape[0]
    if 2 * D > math.comb(L, N):
        raise ValueError("the 2D Ritz vectors need a sector of dimension at least 2D")
    pre = precond.Preconditioner(h, v, N, gamma, prm.c0, prm.c_lower, prm.c_upper, prm.correction)
    mode = prm.truncation

    def trunc(x, eps):
        return precond._trunc(x, L, N, eps, prm.cap, mode)

    eps_num = prm.eps_num if prm.eps_num is not None else 0.5 * (1.0 - prm.c)
    zeta = eps_num / (1.0 + prm.c)
    eta = math.inf
    if X0 is None:
        cols = [fock.determinant(L, occ) for occ in start_determinants(h, N, D)]
    else:
        cols = [X0[:, i].copy() for i in range(D)]
    Phi = np.stack(cols, axis=1)
    hist = []
    s_prev = s_prev2 = None
    for it in range(prm.max_iter):
        # 1. Rayleigh-Ritz on span Phi
        HPhi = np.stack([fock.apply_h(h, v, Phi[:, j], gamma) for j in range(D)], axis=1)
        Hm = Phi.T @ HPhi
        Em = Phi.T @ Phi
        lam, V = _gen_eig_lowest(0.5 * (Hm + Hm.T), 0.5 * (Em + Em.T), D)
        Psi = Phi @ V
        HPsi = HPhi @ V
        # 2. start value of eta_res
        if s_prev is None:
            est = 0.0
            for i in range(D):
                y0 = trunc(HPsi[:, i], 0.0)[0]
                r0 = trunc(y0 - lam[i] * Psi[:, i], 0.0)[0]
                est = max(est, pre.s_max * float(np.linalg.norm(r0)))
        elif s_prev2 is None or s_prev2 <= 0.0:
            est = s_prev
        else:
            est = s_prev * min(1.0, s_prev / s_prev2)
        eta = min(2.0 * eta, 0.8 * zeta * est)
        # 3.-4. residuals and their preconditioned forms
        retries = 0
        while True:
            e12 = eta / (3.0 * pre.s_max)
            S, ns, cap_bound = [], [], False
            for i in range(D):
                y, _, cb1, _, _ = trunc(HPsi[:, i], e12)
                r, _, cb2, _, _ = trunc(y - lam[i] * Psi[:, i], e12)
                s, cb3, _, _ = precond.apply_sorted(pre, r, eta / 3.0, prm.cap, N, mode)
                S.append(s)
                ns.append(float(np.linalg.norm(s)))
                cap_bound = cap_bound or cb1 or cb2 or cb3
            if min(ns) >= (1.0 + 1.0 / zeta) * eta or cap_bound or retries >= prm.max_retries:
                break
            eta *= 0.8
            retries += 1
        rho = [(ns[i] + eta) / (math.sqrt(1.0 - prm.c) * math.sqrt(lam[i])) for i in range(D)]
        bound = bounds.eigvec_error_bound(rho[0], prm.delta)
        rec = dict(it=it, lam=lam.copy(), E=lam - gamma, rho=np.array(rho), bound=bound,
                   s_norm=np.array(ns), eta=eta, retries=retries, cap_bound=bool(cap_bound))
        if bound <= prm.tau:
            rec["stop"] = True
            hist.append(rec)
            return Psi, hist, pre
        # 6. Ritz step on (Psi, P / ||P||)
        P = [precond.apply_sorted(pre, S[i], pre.s_max * eta / 3.0, prm.cap, N, mode)[0] for i in range(D)]
        npn = [float(np.linalg.norm(p)) for p in P]
        if all(n == 0.0 for n in npn):
            rec["stop"] = True
            rec["direction_vanished"] = True
            hist.append(rec)
            return Psi, hist, pre
        if any(n == 0.0 for n in npn):
            raise RuntimeError("a search direction vanished while others did not")
        P = [p / n for p, n in zip(P, npn)]
        Bas = np.concatenate([Psi, np.stack(P, axis=1)], axis=1)
        HBas = np.concatenate([HPsi, np.stack([fock.apply_h(h, v, p, gamma) for p in P], axis=1)], axis=1)
        B = Bas.T @ HBas
        M = Bas.T @ Bas
        lam_s, W = _gen_eig_lowest(0.5 * (B + B.T), 0.5 * (M + M.T), D)
        # 7. truncation tolerance and update
        eta_in = math.inf
        for i in range(D):
            q = math.sqrt(lam_s[i] / (lam_s[i] + prm.t_eig * (lam[i] - lam_s[i])))
            eta_in = min(eta_in, bounds.delta_a(rho[i], q) * math.sqrt(lam_s[i]) / math.sqrt(1.0 + prm.c))
        eta_psi = eta_in * pre.s_min
        Phi = np.stack([trunc(Bas @ W[:, i], eta_psi)[0] for i in range(D)], axis=1)
        rec.update(lam_star=lam_s.copy(), eta_psi=eta_psi)
        hist.append(rec)
        s_prev2, s_prev = s_prev, max(ns)
    return Phi, hist, pre


def run_subspace_joint(h, v, N, gamma, prm: Params, D: int, X0=None):
    """Algorithm 4 with the D columns held jointly (Section 6.2): the same steps as
    ``run_subspace``, with every truncation acting on the joint tensor (the column index as
    one more mode after orbital L, one tolerance for all columns in the Frobenius norm,
    ranks shared): the products H Psi and the residuals R = H Psi - Psi Lambda with e1, e2,
    the sorted S sums with their tolerances (``precond.apply_sorted_joint``), and the update
    Psi <- trunc_{s_min eta_in}(Bas W).  The normalisations Psi <- Phi V and the Ritz
    combinations act on the column index only.  Same records as ``run_subspace``."""
    L = h.shape[0]
    if 2 * D > math.comb(L, N):
        raise ValueError("the 2D Ritz vectors need a sector of dimension at least 2D")
    pre = precond.Preconditioner(h, v, N, gamma, prm.c0, prm.c_lower, prm.c_upper, prm.correction)
    mode = prm.truncation

    def trunc(X, eps):
        Y, _, cb, _ = precond._trunc_joint(X, L, N, eps, prm.cap, mode)
        return Y, cb

    def hmul(X):
        return np.stack([fock.apply_h(h, v, X[:, j], gamma) for j in range(X.shape[1])], axis=1)

    eps_num = prm.eps_num if prm.eps_num is not None else 0.5 * (1.0 - prm.c)
    zeta = eps_num / (1.0 + prm.c)
    eta = math.inf
    if X0 is None:
        Phi = np.stack([fock.determinant(L, occ) for occ in start_determinants(h, N, D)], axis=1)
    else:
        Phi = np.array(X0, dtype=np.float64)
    hist = []
    s_prev = s_prev2 = None
    for it in range(prm.max_iter):
        HPhi = hmul(Phi)
        Hm, Em = Phi.T @ HPhi, Phi.T @ Phi
        lam, V = _gen_eig_lowest(0.5 * (Hm + Hm.T), 0.5 * (Em + Em.T), D)
        Psi, HPsi = Phi @ V, HPhi @ V
        if s_prev is None:
            Y0, _ = trunc(HPsi, 0.0)
            R0, _ = trunc(Y0 - Psi * lam[None, :], 0.0)
            est = pre.s_max * float(np.max(np.linalg.norm(R0, axis=0)))
        elif s_prev2 is None or s_prev2 <= 0.0:
            est = s_prev
        else:
            est = s_prev * min(1.0, s_prev / s_prev2)
        eta = min(2.0 * eta, 0.8 * zeta * est)
        retries = 0
        while True:
            e12 = eta / (3.0 * pre.s_max)
            Y, cb1 = trunc(HPsi, e12)
            R, cb2 = trunc(Y - Psi * lam[None, :], e12)
            S, cb3 = precond.apply_sorted_joint(pre, R, eta / 3.0, prm.cap, N, mode)
            ns = np.linalg.norm(S, axis=0)
            cap_bound = cb1 or cb2 or cb3
            if ns.min() >= (1.0 + 1.0 / zeta) * eta or cap_bound or retries >= prm.max_retries:
                break
            eta *= 0.8
            retries += 1
        rho = [(ns[i] + eta) / (math.sqrt(1.0 - prm.c) * math.sqrt(lam[i])) for i in range(D)]
        bound = bounds.eigvec_error_bound(rho[0], prm.delta)
        rec = dict(it=it, lam=lam.copy(), E=lam - gamma, rho=np.array(rho), bound=bound,
                   s_norm=ns.copy(), eta=eta, retries=retries, cap_bound=bool(cap_bound))
        if bound <= prm.tau:
            rec["stop"] = True
            hist.append(rec)
            return Psi, hist, pre
        P, cb4 = precond.apply_sorted_joint(pre, S, pre.s_max * eta / 3.0, prm.cap, N, mode)
        npn = np.linalg.norm(P, axis=0)
        if np.all(npn == 0.0):
            rec["stop"] = True
            rec["direction_vanished"] = True
            hist.append(rec)
            return Psi, hist, pre
        if np.any(npn == 0.0):
            raise RuntimeError("a search direction vanished while others did not")
        Bas = np.concatenate([Psi, P / npn[None, :]], axis=1)
        HBas = hmul(Bas)
        B, M = Bas.T @ HBas, Bas.T @ Bas
        lam_s, W = _gen_eig_lowest(0.5 * (B + B.T), 0.5 * (M + M.T), D)
        eta_in = math.inf
        for i in range(D):
            q = math.sqrt(lam_s[i] / (lam_s[i] + prm.t_eig * (lam[i] - lam_s[i])))
            eta_in = min(eta_in, bounds.delta_a(rho[i], q) * math.sqrt(lam_s[i]) / math.sqrt(1.0 + prm.c))
        eta_psi = eta_in * pre.s_min
        Phi, cb5 = trunc(Bas @ W, eta_psi)
        rec.update(lam_star=lam_s.copy(), eta_psi=eta_psi, cap_bound=rec["cap_bound"] or bool(cb4 or cb5))
        hist.append(rec)
        s_prev2, s_prev = s_prev, float(ns.max())
    return Phi, hist, pre
