"""Exponential-sum preconditioner S (oracle).

* ``expsum_params`` -- step h and summation range M^-..M^+ (Thm. expsum, eq. expsumparams).
* ``expsum``        -- S(t) = h/sqrt(pi) sum_m e^{mh/2} exp(-e^{mh} t) (eq. expsum).
* ``theta``         -- diagonal approximation theta_i of H + gamma (Section 7.1.1):
                       gamma/N + t_ii + sum_{j=k_i+1}^{k_i+N} (v_ijji - v_ijij),
                       k_i = max(0, i-N), one-based indices.
* ``alpha0``, ``c_const`` -- scaling alpha_0 and constant c of Cor. lrprecond
                       (eqs. Sdef, precondcdef).
* ``terms``         -- S = sum_m alpha_m prod_i diag(1, exp(-beta_m d_i)) with
                       alpha_m = h alpha_0/sqrt(pi) e^{mh/2}, beta_m = e^{mh}/t_min
                       (Section 4.3; beta_m read with 1/t_min, see DESIGN readings)
                       returned as dense diagonals on the 2^L basis.
* ``apply_sorted``  -- the sorted sequential truncated sum of Lemma truncr
                       (Section 5.3.1) applied to the M rank-one diagonal terms.
"""
from __future__ import annotations

import math

import numpy as np

from . import tt


def expsum_params(c0: float, T: float):
    """(h, M_plus, M_minus) of eq. expsumparams."""
    h = math.pi ** 2 / math.log(8.0 * math.sqrt(2.0) / c0 + 1.0)
    lg = abs(math.log(math.sqrt(math.pi) * c0 / 4.0))
    m_plus = math.ceil(math.log(lg) / h)
    m_minus = -math.ceil((2.0 * lg + math.log(T)) / h)
    return h, m_plus, m_minus


def expsum(t, h: float, m_plus: int, m_minus: int):
    t = np.asarray(t, dtype=np.float64)
    m = np.arange(m_minus, m_plus + 1, dtype=np.float64)
    return (h / math.sqrt(math.pi)) * np.sum(
        np.exp(m * h / 2.0)[:, None] * np.exp(-np.exp(m * h)[:, None] * t.reshape(1, -1)),
        axis=0).reshape(t.shape)


def theta(h: np.ndarray, v: np.ndarray, N: int, gamma: float) -> np.ndarray:
    L = h.shape[0]
    th = np.zeros(L)
    for i1 in range(1, L + 1):  # one-based orbital index as in the paper
        k = max(0, i1 - N)
        acc = gamma / N + h[i1 - 1, i1 - 1]
        for j1 in range(k + 1, k + N + 1):
            i, j = i1 - 1, j1 - 1
            acc += v[i, j, j, i] - v[i, j, i, j]
        th[i1 - 1] = acc
    return th


def t_range(th: np.ndarray, N: int):
    """(t_min, t_max): extreme eigenvalues of D = sum theta_i a_i^* a_i on F_N,
    the sums of the N smallest and N largest theta_i."""
    s = np.sort(th)
    return float(s[:N].sum()), float(s[-N:].sum())


def alpha0(t_min: float, c0: float, c_lower: float = 1.0, c_upper: float = 1.0) -> float:
    return math.sqrt(2.0 / (t_min * (c_lower * (1 - c0) ** 2 + c_upper * (1 + c0) ** 2)))


def c_const(c0: float, c_lower: float, c_upper: float) -> float:
    up = c_upper * (1 + c0) ** 2
    lo = c_lower * (1 - c0) ** 2
    return (up - lo) / (up + lo)


class Preconditioner:
    """All scalars of S for one problem."""

    def __init__(self, h, v, N, gamma, c0=0.1, c_lower=1.0, c_upper=1.0, delta=None):
        """delta: None, or an L x (N+1) correction of theta_i per (site, particles on the
        sites before it) (``oracle.learned``); t_min and t_max then follow from the
        corrected diagonal."""
        self.L = h.shape[0]
        self.N = N
        self.th = theta(h, v, N, gamma)
        self.delta = None if delta is None else np.asarray(delta, dtype=np.float64).reshape(self.L, N + 1)
        if self.delta is None:
            self.t_min, self.t_max = t_range(self.th, N)
        else:
            from .learned import t_range as t_range_corrected
            self.t_min, self.t_max = t_range_corrected(self.th, self.delta, N)
        if not self.t_min > 0.0:
            raise ValueError("t_min <= 0: the shift does not make D positive")
        self.T = self.t_max / self.t_min
        self.h, self.m_plus, self.m_minus = expsum_params(c0, self.T)
        self.a0 = alpha0(self.t_min, c0, c_lower, c_upper)
        m = np.arange(self.m_minus, self.m_plus + 1)
        self.alpha = self.h * self.a0 / math.sqrt(math.pi) * np.exp(m * self.h / 2.0)
        self.beta = np.exp(m * self.h) / self.t_min
        # extreme eigenvalues of S on F_N (S(t) decreases in t)
        self.s_max = float(self.a0 * expsum(1.0, self.h, self.m_plus, self.m_minus))
        self.s_min = float(self.a0 * expsum(self.T, self.h, self.m_plus, self.m_minus))

    @property
    def M(self):
        return len(self.alpha)

    def diagonals(self):
        """d_m[beta] = alpha_m prod_{i occupied in beta} exp(-beta_m theta_i), m = 0..M-1."""
        L = self.L
        idx = np.arange(1 << L, dtype=np.int64)
        occ_sum = np.zeros(1 << L)
        left = np.zeros(1 << L, dtype=np.int64)  # particles on the sites before i
        for i in range(L):
            bit = (idx >> i) & 1
            if self.delta is None:
                occ_sum += bit * self.th[i]
            else:
                occ_sum += bit * (self.th[i] + self.delta[i, np.minimum(left, self.N)])
            left += bit
        return [a * np.exp(-b * occ_sum) for a, b in zip(self.alpha, self.beta)]

    def apply_exact(self, x):
        return sum(d * x for d in self.diagonals())


def _trunc(x, L, N, eps, cap, truncation):
    if truncation == "parallel":
        y, rho, cb, m = tt.truncate_parallel(x, L, N, eps, cap)
        return y, rho, cb, m, None
    return tt.truncate(x, L, N, eps, cap)


def apply_sorted(pre: Preconditioner, x: np.ndarray, eta: float, cap: int, N: int,
                 truncation: str = "sequential"):
    """S x by the sorted sequential truncated sum (Lemma truncr and the text after it).

    Terms s_m = S_m x are sorted by norm ascending (equal norms: lower m first); the
    first J0 terms with sum of norms <= eta/3 are dropped; then
    y <- trunc_{eps_j}(y + s_j) with eps_j = eta ||s_j|| / (3 sum_{i>J0} ||s_i||);
    finally y <- trunc_{eta/3}(y).  Returns (y, cap_bound, n_rounds, min_margin)."""
    L = pre.L
    terms = [d * x for d in pre.diagonals()]
    norms = [float(np.linalg.norm(t)) for t in terms]
    order = sorted(range(len(terms)), key=lambda m: (norms[m], m))
    csum = 0.0
    j0 = 0
    for j, m in enumerate(order):
        if csum + norms[m] <= eta / 3.0:
            csum += norms[m]
            j0 = j + 1
        else:
            break
    rest = order[j0:]
    total = sum(norms[m] for m in rest)
    y = np.zeros_like(x)
    cap_bound = False
    margin = math.inf
    rounds = 0
    for m in rest:
        eps_j = eta * norms[m] / (3.0 * total) if total > 0 else 0.0
        y, _, cb, mg, _ = _trunc(y + terms[m], L, N, eps_j, cap, truncation)
        cap_bound |= cb
        margin = min(margin, mg)
        rounds += 1
    y, _, cb, mg, _ = _trunc(y, L, N, eta / 3.0, cap, truncation)
    cap_bound |= cb
    margin = min(margin, mg)
    return y, cap_bound, rounds + 1, margin


def _trunc_joint(X, L, N, eps, cap, truncation):
    if truncation == "parallel":
        return tt.truncate_parallel_joint(X, L, N, eps, cap)
    return tt.truncate_joint(X, L, N, eps, cap)


def apply_sorted_joint(pre: Preconditioner, X: np.ndarray, eta: float, cap: int, N: int,
                       truncation: str = "sequential"):
    """``apply_sorted`` on D columns held jointly (2^L x D): the terms S_m X, their
    Frobenius norms, and every truncation of the sorted sum acting on the joint tensor.
    Returns (Y, cap_bound)."""
    L = pre.L
    terms = [d[:, None] * X for d in pre.diagonals()]
    norms = [float(np.linalg.norm(t)) for t in terms]
    order = sorted(range(len(terms)), key=lambda m: (norms[m], m))
    csum, j0 = 0.0, 0
    for j, m in enumerate(order):
        if csum + norms[m] <= eta / 3.0:
            csum += norms[m]
            j0 = j + 1
        else:
            break
    rest = order[j0:]
    total = sum(norms[m] for m in rest)
    Y = np.zeros_like(X)
    cap_bound = False
    for m in rest:
        eps_j = eta * norms[m] / (3.0 * total) if total > 0 else 0.0
        Y, _, cb, _ = _trunc_joint(Y + terms[m], L, N, eps_j, cap, truncation)
        cap_bound |= cb
    Y, _, cb, _ = _trunc_joint(Y, L, N, eta / 3.0, cap, truncation)
    return Y, cap_bound or cb
