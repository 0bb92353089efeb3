"""Particle-number blocked matricisations and TT-SVD truncation (oracle).

The k-th matricisation of x in F^L_N (rows alpha_1..alpha_k, columns alpha_{k+1}..alpha_L,
Section 2.2) is block diagonal in n = number of particles among orbitals 1..k; the
sector set is K_k = {max(0, N-L+k), ..., min(N, k)} (Section 2.3).  Block n has
C(k,n) rows and C(L-k, N-n) columns.

trunc(x; eps, cap) is the sequential (left to right) TT-SVD truncation: at each cut
k = 1..L-1 the current tensor is projected onto the kept left singular vectors of its
blocked matricisation.  The error bound of eq. ttsvdquasiopt gives
||x - trunc(x)|| <= eps when each cut discards at most (eps/sqrt(L-1))^2 of squared
singular values.  Rank selection across sectors (a reading; the paper has no rank cap):

1. singular values <= zero_tol * sigma_max at this cut are dropped as numerical zeros;
2. the rest are ordered by value, descending; exact ties go to the lower sector n,
   then to the lower index inside the sector;
3. s_tol = the least count whose discarded tail has sum sigma^2 <= (eps/sqrt(L-1))^2;
4. s = min(s_tol, cap), at least 1; "cap bound" is recorded when s_tol > cap.
"""
from __future__ import annotations

import math

import numpy as np

ZERO_TOL = 1e-12
# Numerical-zero level of the simultaneous truncation, whose singular values come from
# Gram matrices (accurate to about sqrt(machine epsilon) of the largest one).
ZERO_TOL_PARALLEL = 1e-6


def sectors(L: int, N: int, k: int):
    return list(range(max(0, N - L + k), min(N, k) + 1))


def _popcount_table(bits: int) -> np.ndarray:
    idx = np.arange(1 << bits, dtype=np.int64)
    return np.array([bin(int(b)).count("1") for b in idx])


def blocks(x: np.ndarray, L: int, N: int, k: int):
    """{n: (left_idx, right_idx, B_n)} for the k-th matricisation, B_n = rows x cols."""
    X = x.reshape(1 << (L - k), 1 << k)  # [right bits, left bits]
    pl = _popcount_table(k)
    pr = _popcount_table(L - k)
    out = {}
    for n in sectors(L, N, k):
        li = np.nonzero(pl == n)[0]
        ri = np.nonzero(pr == N - n)[0]
        out[n] = (li, ri, X[np.ix_(ri, li)].T.copy())
    return out


def select(svals: dict, delta: float, cap: int, zero_tol: float = ZERO_TOL):
    """Kept count per sector from singular values {n: descending array} (rules 1-4).

    Returns (kept: dict n -> int, cap_bound: bool, margin) where margin is the
    relative gap between the last kept and the first discarded value (inf if none),
    used by tests to decide whether the integer decision is well conditioned."""
    allv = [(s, n, j) for n, sv in svals.items() for j, s in enumerate(sv)]
    kept = {n: 0 for n in svals}
    if not allv:
        return kept, False, math.inf
    smax = max(s for s, _, _ in allv)
    if smax <= 0.0:
        return kept, False, math.inf
    cand = [t for t in allv if t[0] > zero_tol * smax]
    cand.sort(key=lambda t: (-t[0], t[1], t[2]))
    sq = np.array([t[0] ** 2 for t in cand])
    tail = np.concatenate([np.cumsum(sq[::-1])[::-1], [0.0]])  # tail[s] = sum_{i>=s}
    s_tol = int(np.argmax(tail <= delta * delta))
    cap_bound = s_tol > cap
    s = max(1, min(s_tol, cap))
    for t in cand[:s]:
        kept[t[1]] += 1
    margin = math.inf
    if s < len(cand):
        margin = (cand[s - 1][0] - cand[s][0]) / smax
    return kept, cap_bound, margin


def select_floor(svals: dict, delta: float, cap: int, zero_tol: float = ZERO_TOL_PARALLEL):
    """``select`` for singular values that are only accurate to a numerical-zero level
    zero_tol * sigma_max (those of the simultaneous truncation, from Gram matrices).
    The values at or below that level are dropped as zeros, as in ``select``; since
    their weight is not known to be zero, the tolerance counts as met only when their
    sum of squares is at most delta^2 as well (for delta > 0; delta = 0 asks for the
    numerically exact truncation).  Otherwise "cap bound" is reported:
    the truncation could not certify its tolerance, which stops the retry loop of
    Algorithm 2 like a binding rank cap."""
    kept, cap_bound, margin = select(svals, delta, cap, zero_tol)
    allv = [s for sv in svals.values() for s in sv]
    if allv:
        smax = max(allv)
        floor2 = sum(s * s for s in allv if s <= zero_tol * smax)
        if smax > 0 and delta > 0 and floor2 > delta * delta:
            cap_bound = True
    return kept, cap_bound, margin


def truncate(x: np.ndarray, L: int, N: int, eps: float, cap: int, zero_tol: float = ZERO_TOL):
    """Sequential TT-SVD truncation.  Returns (y, rho, cap_bound, min_margin, svals).

    rho[k][n] is the kept rank of sector n at cut k (rho[0][0] = rho[L][N] = 1)."""
    delta = eps / math.sqrt(L - 1) if L > 1 else eps
    y = x.copy()
    rho = [dict() for _ in range(L + 1)]
    rho[0] = {0: 1}
    rho[L] = {N: 1}
    cap_bound = False
    min_margin = math.inf
    all_svals = []
    for k in range(1, L):
        bl = blocks(y, L, N, k)
        svd = {}
        sv = {}
        for n, (li, ri, B) in bl.items():
            if B.size == 0:
                svd[n] = (np.zeros((B.shape[0], 0)), np.zeros(0))
                sv[n] = np.zeros(0)
                continue
            U, s, _ = np.linalg.svd(B, full_matrices=False)
            svd[n] = (U, s)
            sv[n] = s
        kept, cb, margin = select(sv, delta, cap, zero_tol)
        cap_bound |= cb
        min_margin = min(min_margin, margin)
        all_svals.append(sv)
        Y = y.reshape(1 << (L - k), 1 << k)
        for n, (li, ri, B) in bl.items():
            U = svd[n][0][:, :kept[n]]
            Bp = U @ (U.T @ B)
            Y[np.ix_(ri, li)] = Bp.T
        y = Y.reshape(-1)
        rho[k] = dict(kept)
    return y, rho, cap_bound, min_margin, all_svals


def ranks(x: np.ndarray, L: int, N: int, zero_tol: float = ZERO_TOL):
    """Numerical rank of every sector block at every cut (rho table of x itself)."""
    rho = [dict() for _ in range(L + 1)]
    rho[0] = {0: 1}
    rho[L] = {N: 1}
    for k in range(1, L):
        bl = blocks(x, L, N, k)
        svs = {n: (np.linalg.svd(B, compute_uv=False) if B.size else np.zeros(0))
               for n, (_, _, B) in bl.items()}
        smax = max([s.max() for s in svs.values() if s.size] + [0.0])
        rho[k] = {n: int(np.sum(s > zero_tol * smax)) for n, s in svs.items()}
    return rho


def singular_values(x: np.ndarray, L: int, N: int, k: int):
    """{n: descending singular values of sector block n at cut k}."""
    return {n: (np.linalg.svd(B, compute_uv=False) if B.size else np.zeros(0))
            for n, (_, _, B) in blocks(x, L, N, k).items()}


def truncate_parallel(x: np.ndarray, L: int, N: int, eps: float, cap: int,
                      zero_tol: float = ZERO_TOL_PARALLEL):
    """Simultaneous truncation y = P_1 P_2 ... P_{L-1} x.

    P_k is the orthogonal projector onto the kept left singular vectors of the k-th
    blocked matricisation of the ORIGINAL x (acting on orbitals 1..k), with the ranks of
    every bond chosen independently by ``select_floor`` with the per-bond tolerance
    eps/sqrt(L-1).  The error splits orthogonally: x - P_1 Y = (I - P_1) x + P_1 (x - Y)
    with Y = P_2 ... P_{L-1} x, the two parts in complementary ranges, so
    ||x - y||^2 <= ||(I - P_1) x||^2 + ||x - Y||^2 <= sum_k ||(I - P_k) x||^2, and each
    term is the discarded tail of bond k: the first inequality of eq. ttsvdquasiopt
    holds for these projectors too, and ||x - y|| <= eps.
    Returns (y, rho, cap_bound, min_margin)."""
    delta = eps / math.sqrt(L - 1) if L > 1 else eps
    rho = [dict() for _ in range(L + 1)]
    rho[0] = {0: 1}
    rho[L] = {N: 1}
    cap_bound = False
    min_margin = math.inf
    proj = {}
    for k in range(1, L):
        bl = blocks(x, L, N, k)
        svd, sv = {}, {}
        for n, (li, ri, B) in bl.items():
            if B.size == 0:
                svd[n] = np.zeros((B.shape[0], 0))
                sv[n] = np.zeros(0)
                continue
            U, s, _ = np.linalg.svd(B, full_matrices=False)
            svd[n], sv[n] = U, s
        kept, cb, margin = select_floor(sv, delta, cap, zero_tol)
        cap_bound |= cb
        min_margin = min(min_margin, margin)
        rho[k] = dict(kept)
        proj[k] = {n: svd[n][:, :kept[n]] for n in bl}
    y = x.copy()
    for k in range(L - 1, 0, -1):
        Y = y.reshape(1 << (L - k), 1 << k)
        for n, (li, ri, B) in blocks(y, L, N, k).items():
            U = proj[k][n]
            Y[np.ix_(ri, li)] = (U @ (U.T @ B)).T
        y = Y.reshape(-1)
    return y, rho, cap_bound, min_margin


# ---------------------------------------------------------------- joint truncation
#
# D columns X (2^L x D) held jointly (Section 6.2, joint tensor parameterisation): the
# column index is one more mode of the tensor, placed after orbital L.  The k-th
# matricisation then has the configurations of orbitals 1..k as rows and those of
# orbitals k+1..L together with the column index as columns; it is block diagonal in the
# particle number n of orbitals 1..k (the index carries none).  Truncations act on the
# joint tensor with one tolerance for all columns (Frobenius norm).


def joint_blocks(X: np.ndarray, L: int, N: int, k: int):
    """{n: (left_idx, right_idx, B_n)}, B_n = rows x (right configs x D)."""
    D = X.shape[1]
    T = X.reshape(1 << (L - k), 1 << k, D)  # [right bits, left bits, column]
    pl = _popcount_table(k)
    pr = _popcount_table(L - k)
    out = {}
    for n in sectors(L, N, k):
        li = np.nonzero(pl == n)[0]
        ri = np.nonzero(pr == N - n)[0]
        B = np.transpose(T[np.ix_(ri, li, np.arange(D))], (1, 0, 2)).reshape(len(li), len(ri) * D)
        out[n] = (li, ri, B.copy())
    return out


def _put_joint(X, L, k, li, ri, B):
    D = X.shape[1]
    T = X.reshape(1 << (L - k), 1 << k, D)
    T[np.ix_(ri, li, np.arange(D))] = np.transpose(B.reshape(len(li), len(ri), D), (1, 0, 2))


def truncate_joint(X: np.ndarray, L: int, N: int, eps: float, cap: int, zero_tol: float = ZERO_TOL):
    """Sequential TT-SVD truncation of the joint tensor (``truncate`` with the column index
    as the last mode): ||X - Y||_F <= eps, ranks shared by all columns.
    Returns (Y, rho, cap_bound, min_margin)."""
    delta = eps / math.sqrt(L - 1) if L > 1 else eps
    Y = X.copy()
    rho = [dict() for _ in range(L + 1)]
    rho[0] = {0: 1}
    rho[L] = {N: X.shape[1]}
    cap_bound, min_margin = False, math.inf
    for k in range(1, L):
        bl = joint_blocks(Y, L, N, k)
        svd, sv = {}, {}
        for n, (li, ri, B) in bl.items():
            if B.size == 0:
                svd[n], sv[n] = np.zeros((B.shape[0], 0)), np.zeros(0)
                continue
            U, s, _ = np.linalg.svd(B, full_matrices=False)
            svd[n], sv[n] = U, s
        kept, cb, margin = select(sv, delta, cap, zero_tol)
        cap_bound |= cb
        min_margin = min(min_margin, margin)
        for n, (li, ri, B) in bl.items():
            U = svd[n][:, :kept[n]]
            _put_joint(Y, L, k, li, ri, U @ (U.T @ B))
        rho[k] = dict(kept)
    return Y, rho, cap_bound, min_margin


def truncate_parallel_joint(X: np.ndarray, L: int, N: int, eps: float, cap: int,
                            zero_tol: float = ZERO_TOL_PARALLEL):
    """``truncate_parallel`` of the joint tensor: P_1 ... P_{L-1} X with P_k from the k-th
    joint matricisation of X itself, tolerance eps/sqrt(L-1) per bond (``select_floor``).
    Returns (Y, rho, cap_bound, min_margin)."""
    delta = eps / math.sqrt(L - 1) if L > 1 else eps
    rho = [dict() for _ in range(L + 1)]
    rho[0] = {0: 1}
    rho[L] = {N: X.shape[1]}
    cap_bound, min_margin = False, math.inf
    proj = {}
    for k in range(1, L):
        bl = joint_blocks(X, L, N, k)
        svd, sv = {}, {}
        for n, (li, ri, B) in bl.items():
            if B.size == 0:
                svd[n], sv[n] = np.zeros((B.shape[0], 0)), np.zeros(0)
                continue
            U, s, _ = np.linalg.svd(B, full_matrices=False)
            svd[n], sv[n] = U, s
        kept, cb, margin = select_floor(sv, delta, cap, zero_tol)
        cap_bound |= cb
        min_margin = min(min_margin, margin)
        rho[k] = dict(kept)
        proj[k] = {n: svd[n][:, :kept[n]] for n in bl}
    Y = X.copy()
    for k in range(L - 1, 0, -1):
        for n, (li, ri, B) in joint_blocks(Y, L, N, k).items():
            U = proj[k][n]
            _put_joint(Y, L, k, li, ri, U @ (U.T @ B))
    return Y, rho, cap_bound, min_margin
