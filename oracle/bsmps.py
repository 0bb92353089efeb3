"""Block-sparse MPS oracle (O-MPS).  TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke entry point and the benchmark's CPU-baseline leg may use
this module; the GPU library shares no code with it.  Plain float64 NumPy, written for
checking by eye rather than for speed.

Unlike the dense oracle (``fock``, ``tt``), which holds every state as its 2^L-vector,
this one holds states as particle-number block-sparse MPS (Section 2.3, eq.
blockstructure): site k has, for each left sector n in K_{k-1}, an unoccupied block
U_{k,n} (rho[k-1][n] x rho[k][n]) and an occupied block O_{k,n}
(rho[k-1][n] x rho[k][n+1]).  It therefore reaches the workload sizes (L = 24 and
beyond) and gives the operator application with a finite intermediate rank m_zip a
definition of its own.

Contents, each pinned in ``tests/test_oracle_bsmps.py`` against the dense oracle or an
identity of its own:

* ``build_mpo``     -- matrix product operator of H = sum h_ij a_i^* a_j
                       + sum w_ijkl a_i^* a_j^* a_k a_l (eq. hamil, antisymmetrised
                       two-body part, Thm. opranks), built from the Kronecker factors of
                       every term (eq. anniloperator).  See its docstring for the bond
                       states.
* ``dot``, ``lincomb``, ``scale`` -- transfer sweep; addition as concatenation
                       (Section 2.3).
* ``truncate``      -- sequential TT-SVD truncation trunc_eps with a rank cap
                       (Section 2.2, eq. ttsvdquasiopt), ranks chosen across sectors
                       by ``tt.select``.
* ``truncate_parallel`` -- the simultaneous truncation P_1 ... P_{L-1} x (each P_k the
                       projector onto the kept left singular vectors of the k-th
                       matricisation of x, tolerance eps/sqrt(L-1) per bond).
* ``zipup``, ``apply_h`` -- H x applied site by site (the matrix-free product of
                       Section 2.4) with an intermediate rank m_zip: at every site the
                       partially contracted panel is factorised and only its m_zip
                       leading left singular vectors are kept.  m_zip <= 0 keeps every
                       non-zero singular value, which is H x itself.  Then trunc.
* ``expect``        -- <a|H|b> by an environment sweep (eq. exactrq).
* ``apply_s``       -- S x by the sorted sequential truncated sum of Lemma truncr on the
                       rank-one terms of Section 4.3.
* ``run``           -- Algorithm 2 in the physical variable psi = S x, step for step as
                       ``pinvit.run`` but on block-sparse MPS and with m_zip.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import bounds, precond, tt
from .mps import block_shapes, to_dense as _dense_of_export, unpack
from .tt import sectors

# ---------------------------------------------------------------- block-sparse MPS


def _svd(M):
    """Thin SVD.  LAPACK's divide-and-conquer driver (NumPy's) now and then reports
    non-convergence on strongly graded blocks; the QR-iteration driver then computes
    the same factorisation."""
    try:
        return np.linalg.svd(M, full_matrices=False)
    except np.linalg.LinAlgError:
        return scipy.linalg.svd(M, full_matrices=False, lapack_driver="gesvd")


def _valid(L, N, k, n):
    return max(0, N - L + k) <= n <= min(N, k)


class BMps:
    """Block-sparse MPS.  ``blk[k][(n, s)]`` (k = 1..L; index 0 unused) is the block of
    site k with left sector n and occupation s of orbital k: the U block for s = 0, the O
    block for s = 1.  ``rho`` is the (L+1) x (N+1) block table."""

    def __init__(self, L, N, rho, blk):
        self.L, self.N = L, N
        self.rho = np.asarray(rho, dtype=np.int64).copy()
        self.blk = blk
        for k in range(1, L + 1):
            for (n, s), b in blk[k].items():
                assert b.shape == (self.rho[k - 1][n], self.rho[k][n + s]), (k, n, s, b.shape)

    def copy(self):
        return BMps(self.L, self.N, self.rho, [None] + [{key: b.copy() for key, b in self.blk[k].items()}
                                                        for k in range(1, self.L + 1)])

    def max_rank(self):
        return int(max(self.rho[k].sum() for k in range(self.L + 1)))

    def keys(self, k):
        """(n, s) of the blocks of site k in export order."""
        L, N = self.L, self.N
        out = []
        for n in sectors(L, N, k - 1):
            for s in (0, 1):
                if _valid(L, N, k, n + s):
                    out.append((n, s))
        return out


def empty_rho(L, N):
    rho = np.zeros((L + 1, N + 1), dtype=np.int64)
    rho[0][0] = 1
    rho[L][N] = 1
    return rho


def from_blocks(L, N, blk):
    """BMps from blocks alone: the block table is read off their shapes."""
    rho = empty_rho(L, N)
    for k in range(1, L + 1):
        for (n, s), b in blk[k].items():
            rho[k - 1][n] = b.shape[0]
            rho[k][n + s] = b.shape[1]
    return BMps(L, N, rho, blk)


def from_export(L, N, rho, data):
    """The library's export layout (see ``oracle.mps``) as a BMps."""
    ub = unpack(L, N, rho, data)
    blk = [None] + [dict() for _ in range(L)]
    for (k, n, kind), b in ub.items():
        blk[k][(n, kind)] = np.array(b, dtype=np.float64)
    return BMps(L, N, rho, blk)


def to_export(x: BMps):
    """(rho, data) in the export layout."""
    parts = []
    for k, n, kind, r, c in block_shapes(x.L, x.N, x.rho):
        parts.append(x.blk[k][(n, kind)].T.reshape(-1))
    data = np.concatenate(parts) if parts else np.zeros(0)
    return x.rho.astype(np.int32), data


def to_dense(x: BMps) -> np.ndarray:
    """The 2^L-vector of x (eq. mps), for small L."""
    rho, data = to_export(x)
    if any(x.rho[k].sum() == 0 for k in range(x.L + 1)):
        return np.zeros(1 << x.L)
    return _dense_of_export(x.L, x.N, rho, data)


def determinant(L, N, occupied):
    """Rank-one MPS of the Slater determinant with the given zero-based orbitals."""
    occ = set(int(i) for i in occupied)
    assert len(occ) == N
    rho = np.zeros((L + 1, N + 1), dtype=np.int64)
    n = 0
    rho[0][0] = 1
    path = [0]
    for k in range(1, L + 1):
        n += (k - 1) in occ
        path.append(n)
        rho[k][n] = 1
    blk = [None] + [dict() for _ in range(L)]
    for k in range(1, L + 1):
        for n in sectors(L, N, k - 1):
            for s in (0, 1):
                if _valid(L, N, k, n + s):
                    blk[k][(n, s)] = np.zeros((rho[k - 1][n], rho[k][n + s]))
        s = int((k - 1) in occ)
        blk[k][(path[k - 1], s)][0, 0] = 1.0
    return BMps(L, N, rho, blk)


def scale(x: BMps, a: float) -> BMps:
    y = x.copy()
    for key in y.blk[1]:
        y.blk[1][key] *= a
    return y


def dot(a: BMps, b: BMps) -> float:
    """<a, b> by the transfer sweep E_k[m] = sum_{n+s=m} A_{k,n,s}^T E_{k-1}[n] B_{k,n,s}."""
    L, N = a.L, a.N
    E = {0: np.ones((1, 1))}
    for k in range(1, L + 1):
        nxt = {}
        for (n, s), A in a.blk[k].items():
            if n not in E:
                continue
            B = b.blk[k][(n, s)]
            t = A.T @ E[n] @ B
            m = n + s
            nxt[m] = nxt[m] + t if m in nxt else t
        E = nxt
    return float(E[N][0, 0]) if N in E else 0.0


def norm(x: BMps) -> float:
    return math.sqrt(max(dot(x, x), 0.0))


def lincomb(a: float, x: BMps, b: float, y: BMps) -> BMps:
    """a x + b y by concatenation (Section 2.3): first cores side by side, last cores
    stacked, inner cores block diagonal; block tables add on the inner bonds."""
    L, N = x.L, x.N
    rho = x.rho + y.rho
    rho[0][0] = 1
    rho[L][N] = 1
    blk = [None] + [dict() for _ in range(L)]
    for k in range(1, L + 1):
        for key in x.blk[k]:
            X, Y = x.blk[k][key], y.blk[k][key]
            if L == 1:
                blk[k][key] = a * X + b * Y
            elif k == 1:
                blk[k][key] = np.hstack([a * X, b * Y])
            elif k == L:
                blk[k][key] = np.vstack([X, Y])
            else:
                Z = np.zeros((X.shape[0] + Y.shape[0], X.shape[1] + Y.shape[1]))
                Z[:X.shape[0], :X.shape[1]] = X
                Z[X.shape[0]:, X.shape[1]:] = Y
                blk[k][key] = Z
    return BMps(L, N, rho, blk)


# ---------------------------------------------------------------- orthogonalisation and truncation


def right_orthogonalize(x: BMps, zero_tol: float = tt.ZERO_TOL) -> BMps:
    """Sites L..2 made right-orthogonal: per left sector n of site k the matrix
    C = [U_{k,n} | O_{k,n}] = U S V^T (SVD), the rows V^T (those with sigma above
    zero_tol times the largest sigma of the bond) become the new blocks and U S is
    multiplied into the blocks of site k-1 that end in sector n."""
    L, N = x.L, x.N
    y = x.copy()
    for k in range(L, 1, -1):
        svd = {}
        smax = 0.0
        for n in sectors(L, N, k - 1):
            parts = [y.blk[k][(n, s)] for s in (0, 1) if (n, s) in y.blk[k]]
            C = np.hstack(parts)
            if C.size == 0:
                svd[n] = (np.zeros((C.shape[0], 0)), np.zeros(0), np.zeros((0, C.shape[1])))
                continue
            U, S, Vt = _svd(C)
            svd[n] = (U, S, Vt)
            if S.size:
                smax = max(smax, S[0])
        for n in sectors(L, N, k - 1):
            U, S, Vt = svd[n]
            r = int(np.sum(S > zero_tol * smax)) if smax > 0 else 0
            y.rho[k - 1][n] = r
            off = 0
            for s in (0, 1):
                if (n, s) in y.blk[k]:
                    w = y.blk[k][(n, s)].shape[1]
                    y.blk[k][(n, s)] = Vt[:r, off:off + w].copy()
                    off += w
            R = U[:, :r] * S[:r]
            for (m, s), B in list(y.blk[k - 1].items()):
                if m + s == n:
                    y.blk[k - 1][(m, s)] = B @ R
    return y


def _left_fused(y: BMps, k: int, n: int):
    """Rows of the left-fused matrix of site k for right sector n: [U_{k,n}; O_{k,n-1}]
    (each part present when its left sector exists); returns (M, [(left n, s, rows)])."""
    parts, rows = [], []
    for s in (0, 1):
        key = (n - s, s)
        if key in y.blk[k]:
            parts.append(y.blk[k][key])
            rows.append((n - s, s, y.blk[k][key].shape[0]))
    M = np.vstack(parts) if parts else np.zeros((0, y.rho[k][n]))
    return M, rows


def truncate(x: BMps, eps: float, cap: int, zero_tol: float = tt.ZERO_TOL):
    """trunc_eps(x) with rank cap, sequential TT-SVD (Section 2.2, eq. ttsvdquasiopt):
    right-orthogonalise, then for k = 1..L-1 factor the left-fused blocks of site k,
    M_n = U S V^T per right sector n, choose the kept counts across sectors with
    per-bond tolerance eps/sqrt(L-1) (``tt.select``), keep U[:, :s] as the new blocks
    and multiply (S V^T)[:s] into site k+1.  Returns (y, cap_bound, min_margin, svals);
    y is left-orthogonal with its norm in the last core."""
    L, N = x.L, x.N
    delta = eps / math.sqrt(L - 1) if L > 1 else eps
    y = right_orthogonalize(x)
    cap_bound = False
    min_margin = math.inf
    all_sv = []
    for k in range(1, L):
        svd, sv, rows = {}, {}, {}
        for n in sectors(L, N, k):
            M, rows[n] = _left_fused(y, k, n)
            if M.size == 0:
                svd[n] = (np.zeros((M.shape[0], 0)), np.zeros(0), np.zeros((0, M.shape[1])))
                sv[n] = np.zeros(0)
                continue
            svd[n] = _svd(M)
            sv[n] = svd[n][1]
        kept, cb, margin = tt.select(sv, delta, cap, zero_tol)
        cap_bound |= cb
        min_margin = min(min_margin, margin)
        all_sv.append(sv)
        for n in sectors(L, N, k):
            U, S, Vt = svd[n]
            s = kept[n]
            y.rho[k][n] = s
            off = 0
            for (m, ss, r) in rows[n]:
                y.blk[k][(m, ss)] = U[off:off + r, :s].copy()
                off += r
            SV = S[:s, None] * Vt[:s]
            for (m, ss), B in list(y.blk[k + 1].items()):
                if m == n:
                    y.blk[k + 1][(m, ss)] = SV @ B
    return y, cap_bound, min_margin, all_sv


def _left_factors(x: BMps):
    """R_k per bond k = 1..L-1 and sector: A_k = Q_k R_k with Q_k orthonormal columns,
    A_k the left part of x at cut k (sites 1..k), by a left-to-right sweep of SVDs."""
    L, N = x.L, x.N
    R = {0: {0: np.ones((1, 1))}}
    for k in range(1, L):
        R[k] = {}
        for n in sectors(L, N, k):
            parts = []
            for s in (0, 1):
                key = (n - s, s)
                if key in x.blk[k]:
                    parts.append(R[k - 1][n - s] @ x.blk[k][key])
            M = np.vstack(parts)
            if M.size == 0:
                R[k][n] = np.zeros((0, M.shape[1]))
                continue
            _, S, Vt = _svd(M)
            R[k][n] = S[:, None] * Vt
    return R


def _right_factors(x: BMps):
    """R'_k per bond k = 1..L-1 and sector: B_k = R'_k Q'_k with Q'_k orthonormal rows,
    B_k the right part of x at cut k (sites k+1..L), by a right-to-left sweep."""
    L, N = x.L, x.N
    R = {L: {N: np.ones((1, 1))}}
    for k in range(L - 1, 0, -1):
        R[k] = {}
        for n in sectors(L, N, k):
            parts = []
            for s in (0, 1):
                if (n, s) in x.blk[k + 1]:
                    parts.append(x.blk[k + 1][(n, s)] @ R[k + 1][n + s])
            M = np.hstack(parts)
            if M.size == 0:
                R[k][n] = np.zeros((M.shape[0], 0))
                continue
            U, S, _ = _svd(M)
            R[k][n] = U * S
    return R


def truncate_parallel(x: BMps, eps: float, cap: int, zero_tol: float = tt.ZERO_TOL_PARALLEL):
    """Simultaneous truncation y = P_1 P_2 ... P_{L-1} x (``tt.truncate_parallel`` on
    block-sparse MPS).  With A_k = Q_k R_k and B_k = R'_k Q'_k the singular values of the
    k-th matricisation are those of C_k = R_k R'_k = U S V^T (per sector); ranks as
    ``tt.select_floor`` with tolerance eps/sqrt(L-1) per bond.  The bond matrices
    L_k = R'_k V_s S_s^{-1} and T_k = U_s^T R_k satisfy A_k L_k T_k = P_k A_k, so the
    cores T_{k-1} x_k L_k of y apply every projector (bonds right to left, each seeing
    the unchanged left part of x).  Returns (y, cap_bound, min_margin)."""
    L, N = x.L, x.N
    delta = eps / math.sqrt(L - 1) if L > 1 else eps
    RL, RR = _left_factors(x), _right_factors(x)
    Lm, Tm = {0: {0: np.ones((1, 1))}}, {0: {0: np.ones((1, 1))}}
    Lm[L], Tm[L] = {N: np.ones((1, 1))}, {N: np.ones((1, 1))}
    rho = empty_rho(L, N)
    cap_bound = False
    min_margin = math.inf
    for k in range(1, L):
        svd, sv = {}, {}
        for n in sectors(L, N, k):
            C = RL[k][n] @ RR[k][n]
            if C.size == 0:
                svd[n] = (np.zeros((C.shape[0], 0)), np.zeros(0), np.zeros((0, C.shape[1])))
                sv[n] = np.zeros(0)
                continue
            svd[n] = _svd(C)
            sv[n] = svd[n][1]
        kept, cb, margin = tt.select_floor(sv, delta, cap, zero_tol)
        cap_bound |= cb
        min_margin = min(min_margin, margin)
        Lm[k], Tm[k] = {}, {}
        for n in sectors(L, N, k):
            U, S, Vt = svd[n]
            s = kept[n]
            rho[k][n] = s
            Lm[k][n] = RR[k][n] @ Vt[:s].T / S[:s]
            Tm[k][n] = U[:, :s].T @ RL[k][n]
    blk = [None] + [dict() for _ in range(L)]
    for k in range(1, L + 1):
        for (n, s), X in x.blk[k].items():
            blk[k][(n, s)] = Tm[k - 1][n] @ X @ Lm[k][n + s]
    return BMps(L, N, rho, blk), cap_bound, min_margin


def trunc(x: BMps, eps: float, cap: int, mode: str = "sequential"):
    """(y, cap_bound) of the truncation of the given mode."""
    if mode == "parallel":
        y, cb, _ = truncate_parallel(x, eps, cap)
        return y, cb
    y, cb, _, _ = truncate(x, eps, cap)
    return y, cb


# ---------------------------------------------------------------- matrix product operator

class Mpo:
    """Sites m = 0..L-1 (orbital m+1).  ``q[m]``: charge of every bond state at cut m
    (ascending); ``blocks[m][(q_in, q_out, s_out, s_in)]``: dense matrix over the states
    of charge q_in at cut m (rows) and of charge q_out at cut m+1 (columns); ``keys[m]``
    the state codes of ``_cut_states`` (for inspection)."""

    def __init__(self, L, q, blocks, keys):
        self.L, self.q, self.blocks, self.keys = L, q, blocks, keys

    def w(self, m):
        return len(self.q[m])

    def wq(self, m, q):
        return int(np.sum(self.q[m] == q))

    def dense_site(self, m):
        """W[b, b', s_out, s_in] (for small tests)."""
        wi, wo = self.w(m), self.w(m + 1)
        W = np.zeros((wi, wo, 2, 2))
        oi = {q: np.nonzero(self.q[m] == q)[0] for q in range(-2, 3)}
        oo = {q: np.nonzero(self.q[m + 1] == q)[0] for q in range(-2, 3)}
        for (qi, qo, so, si), B in self.blocks[m].items():
            W[np.ix_(oi[qi], oo[qo], [so], [si])] = B[:, :, None, None]
        return W

    def to_dense(self):
        """Dense 2^L x 2^L matrix (bit i = orbital i+1), for L <= 8."""
        ops = [np.ones((1, 1))]
        for m in range(self.L):
            W = self.dense_site(m)
            d = ops[0].shape[0]
            nxt = [np.zeros((2 * d, 2 * d)) for _ in range(W.shape[1])]
            for b in range(W.shape[0]):
                for bp in range(W.shape[1]):
                    f = W[b, bp]
                    if not f.any():
                        continue
                    # orbital m+1 is the most significant bit of the new index
                    nxt[bp] += np.kron(f, ops[b])
            ops = nxt
        return ops[0]


def _term_arrays(h, v, shift):
    """The terms of H + shift sum_i n_i as arrays, in product order: h_ij a_i^* a_j for all
    (i, j) (row-major), then w_ijkl a_i^* a_j^* a_k a_l for i < j, k < l (pairs row-major,
    the created pair outer) with w_ijkl = v_ijkl - v_jikl - v_ijlk + v_jilk (the two-body
    sum of eq. hamil antisymmetrised); exact zeros are skipped.  Returns (coef (T,),
    cre (T, 4) bool: creator in that slot, pos (T, 4): orbital, -1 for an empty slot)."""
    L = h.shape[0]
    h1 = h + shift * np.eye(L)
    i1, j1 = np.nonzero(h1 != 0.0)
    w = v - v.transpose(1, 0, 2, 3) - v.transpose(0, 1, 3, 2) + v.transpose(1, 0, 3, 2)
    pi, pj = np.triu_indices(L, 1)
    w2 = w[pi[:, None], pj[:, None], pi[None, :], pj[None, :]]  # [created pair, annihilated pair]
    a2, b2 = np.nonzero(w2 != 0.0)
    coef = np.concatenate([h1[i1, j1], w2[a2, b2]])
    n1, n2 = len(i1), len(a2)
    pos = np.full((n1 + n2, 4), -1, dtype=np.int64)
    pos[:n1, 0], pos[:n1, 1] = i1, j1
    pos[n1:, 0], pos[n1:, 1], pos[n1:, 2], pos[n1:, 3] = pi[a2], pj[a2], pi[b2], pj[b2]
    cre = np.zeros((n1 + n2, 4), dtype=bool)
    cre[:n1, 0] = True
    cre[n1:, 0] = cre[n1:, 1] = True
    return coef, cre, pos


_KIND_I, _KIND_F, _KIND_L, _KIND_R = 0, 1, 2, 3


def _cut_states(cre, pos, m, L):
    """Bond state of every term at cut m (orbitals < m on the left), as (kind, code, charge).
    kind 'I': no operator on the left yet; 'F': all of them on the left; otherwise the
    term is keyed by the operators on the side with fewer of them (on a tie: the left side
    when 2m < L, else the right side), kind 'L' (left operators) or 'R' (right ones).
    The key's operators (at most two: the two-body terms have four) in product order,
    each as 1 + creator * L + orbital, give the code; the charge is the change of the
    particle number that the term's operators left of the cut make."""
    valid = pos >= 0
    left = valid & (pos < m)
    nl = left.sum(axis=1)
    nr = valid.sum(axis=1) - nl
    kind = np.where(nl == 0, _KIND_I, np.where(nr == 0, _KIND_F,
                    np.where((nl < nr) | ((nl == nr) & (2 * m < L)), _KIND_L, _KIND_R)))
    keyop = np.where((kind == _KIND_L)[:, None], left, np.where((kind == _KIND_R)[:, None], valid & ~left, False))
    e = np.where(keyop, 1 + cre * L + pos, 0)
    rank = np.cumsum(keyop, axis=1)  # 1 for the key's first operator, 2 for its second
    if np.any(rank[:, -1] > 2):
        raise RuntimeError("a bond key holds more than two operators")
    first = (e * (keyop & (rank == 1))).sum(axis=1)
    second = (e * (keyop & (rank == 2))).sum(axis=1)
    base = 2 * L + 1
    code = (kind * base + first) * base + second
    dq = (np.where(cre, 1, -1) * left).sum(axis=1)
    return kind, code, dq


def _site_factors(cre, pos, m):
    """(T, 2, 2), entry [s_out, s_in]: factor of every term's Kronecker product on site m,
    the ordered product over its operators of S (orbital above m), a or a^* (orbital m),
    I (below m or no operator): a_p = S x .. x S (sites < p) x A (site p) x I (sites > p),
    eq. anniloperator."""
    T = pos.shape[0]
    f00, f01, f10, f11 = np.ones(T), np.zeros(T), np.zeros(T), np.ones(T)
    for slot in range(4):
        p, c = pos[:, slot], cre[:, slot]
        at = p == m
        # entries of g: I = [[1,0],[0,1]], S = [[1,0],[0,-1]], a = [[0,1],[0,0]], a^* = [[0,0],[1,0]]
        g00 = np.where(at, 0.0, 1.0)
        g01 = (at & ~c).astype(np.float64)
        g10 = (at & c).astype(np.float64)
        g11 = np.where(at, 0.0, np.where(p > m, -1.0, 1.0))
        f00, f01, f10, f11 = (f00 * g00 + f01 * g10, f00 * g01 + f01 * g11,
                              f10 * g00 + f11 * g10, f10 * g01 + f11 * g11)
    return np.stack([np.stack([f00, f01], axis=1), np.stack([f10, f11], axis=1)], axis=1)


def build_mpo(h, v, shift=0.0):
    """MPO of H + shift sum_i n_i (shift = gamma/N gives H + gamma on F_N).

    Every term is c * (x)_m f(m) with the site factors f(m) of ``_site_factors``.  Its bond
    state at cut m is given by ``_cut_states``; the states of a cut are those of all terms,
    ordered by (charge, code).  Along the cuts a term's state is left-type ('I', 'L') up
    to one site and right-type ('R', 'F') after it; on that site its coefficient enters:
    W[b, b'] += c r f(m).  On every other site the entry W[b, b'] is shared by all terms
    with that pair of states: it is the factor of the first such term (in term order),
    and each other term's factor equals it up to a sign; r is the product of those signs
    over the term's other sites.  A left-type state fixes the states before it (its key
    holds the operators left of the cut) and a right-type one those after it, so every
    path through the MPO is the path of whole terms and the MPO equals
    sum_t c_t (x)_m f_t(m)."""
    L = h.shape[0]
    coef, cre, pos = _term_arrays(h, v, shift)
    T = len(coef)
    qs, keys, idx_prev, lt_prev = [], [], None, None
    rsign = np.ones(T)
    mstar = np.full(T, -1)
    b_in = np.zeros(T, dtype=np.int64)
    b_out = np.zeros(T, dtype=np.int64)
    f_trans = np.zeros((T, 2, 2))
    blocks = []
    for m in range(L + 1):
        kind, code, dq = _cut_states(cre, pos, m, L)
        uc, first, inv = np.unique(code, return_index=True, return_inverse=True)
        uq = dq[first]
        order = np.lexsort((uc, uq))          # states by (charge, code)
        rank = np.empty_like(order)
        rank[order] = np.arange(len(order))
        idx = rank[inv]
        qs.append(uq[order])
        keys.append(uc[order])
        lt = (kind == _KIND_I) | (kind == _KIND_L)
        if m == 0 and not np.all(kind == _KIND_I):
            raise RuntimeError("a term has an operator left of the chain")
        if m > 0:
            site = m - 1
            f = _site_factors(cre, pos, site)
            trans = lt_prev & ~lt
            if np.any(trans & (mstar >= 0)) or np.any(~lt_prev & lt):
                raise RuntimeError("a term's state returns to the left type")
            mstar[trans] = site
            b_in[trans], b_out[trans] = idx_prev[trans], idx[trans]
            f_trans[trans] = f[trans]
            # shared entries: pairs of states of the non-transition terms
            nt = np.nonzero(~trans)[0]
            wo = len(keys[m])
            pc = idx_prev[nt] * wo + idx[nt]
            up, pfirst, pinv = np.unique(pc, return_index=True, return_inverse=True)
            canon = f[nt][pfirst]
            ft = f[nt]
            same = np.all(ft == canon[pinv], axis=(1, 2))
            flip = np.all(ft == -canon[pinv], axis=(1, 2))
            if not np.all(same | flip):
                raise RuntimeError(f"shared MPO entry differs by more than a sign at site {site}")
            rsign[nt[flip]] *= -1.0
            blocks.append([(up // wo, up % wo, canon)])
        idx_prev, lt_prev = idx, lt
    if np.any(mstar < 0):
        raise RuntimeError("a term never enters its coefficient")
    # transition entries: c r f(m*) summed over the terms with the same site and states
    val = (coef * rsign)[:, None, None] * f_trans
    for site in range(L):
        sel = np.nonzero(mstar == site)[0]
        if len(sel) == 0:
            continue
        wo = len(keys[site + 1])
        pc = b_in[sel] * wo + b_out[sel]
        up, pinv = np.unique(pc, return_inverse=True)
        acc = np.zeros((len(up), 2, 2))
        np.add.at(acc, pinv, val[sel])
        blocks[site].append((up // wo, up % wo, acc))
    # charge blocks (q_in, q_out, s_out, s_in) -> dense (w_q_in x w_q_out)
    out = []
    for site in range(L):
        qi_all, qo_all = qs[site], qs[site + 1]
        pos_in = np.zeros(len(qi_all), dtype=np.int64)
        pos_out = np.zeros(len(qo_all), dtype=np.int64)
        for q in range(-2, 3):
            pos_in[qi_all == q] = np.arange(int(np.sum(qi_all == q)))
            pos_out[qo_all == q] = np.arange(int(np.sum(qo_all == q)))
        bl = {}
        for b, bp, F in blocks[site]:
            for so in (0, 1):
                for si in (0, 1):
                    val_e = F[:, so, si]
                    nz = np.nonzero(val_e != 0.0)[0]
                    if len(nz) == 0:
                        continue
                    qi, qo = qi_all[b[nz]], qo_all[bp[nz]]
                    if np.any(qo - qi != so - si):
                        raise RuntimeError("MPO entry violates particle-number conservation")
                    for q_in in np.unique(qi):
                        sel = nz[qi == q_in]
                        q_out = int(q_in) + so - si
                        key = (int(q_in), q_out, so, si)
                        if key not in bl:
                            bl[key] = np.zeros((int(np.sum(qi_all == q_in)), int(np.sum(qo_all == q_out))))
                        np.add.at(bl[key], (pos_in[b[sel]], pos_out[bp[sel]]), val_e[sel])
        out.append(bl)
    return Mpo(L, qs, out, keys)


# ---------------------------------------------------------------- operator application


def _site_products(mpo: Mpo, m: int, C: dict, x: BMps, k: int):
    """One site of a sweep.  C[(n, q)] has shape (rho_bra(n), w_q, rho_x(n - q)): the bra
    (or new) sector n, the operator charge q and the ket sector n - q at cut k-1.  Returns
    T2[(n, s_out, q')] = sum over q, s_in of W[q -> q'; s_out, s_in] applied to
    C[(n, q)] contracted with the ket block x_k[(n - q, s_in)], of shape
    (rho_bra(n), w_q', rho_x(k, n + s_out - q'))."""
    T2 = {}
    for (n, q), Cb in C.items():
        for s_in in (0, 1):
            xkey = (n - q, s_in)
            if xkey not in x.blk[k]:
                continue
            T1 = np.tensordot(Cb, x.blk[k][xkey], axes=([2], [0]))  # (a, w_q, c')
            for s_out in (0, 1):
                qo = q + s_out - s_in
                W = mpo.blocks[m].get((q, qo, s_out, s_in))
                if W is None:
                    continue
                t = np.tensordot(T1, W, axes=([1], [0])).transpose(0, 2, 1)  # (a, w_q', c')
                key = (n, s_out, qo)
                T2[key] = T2[key] + t if key in T2 else t
    return T2


def expect(bra: BMps, ket: BMps, mpo: Mpo) -> float:
    """<bra| H |ket> by the environment sweep E_k[(n', q')] = sum_{s_out}
    bra_k[(n'-s_out, s_out)]^T T2[(n'-s_out, s_out, q')] (eq. exactrq with one term)."""
    L, N = ket.L, ket.N
    E = {(0, 0): np.ones((1, 1, 1))}
    for k in range(1, L + 1):
        T2 = _site_products(mpo, k - 1, E, ket, k)
        nxt = {}
        for (n, s_out, qo), t in T2.items():
            bkey = (n, s_out)
            if bkey not in bra.blk[k]:
                continue
            e = np.tensordot(bra.blk[k][bkey], t, axes=([0], [0]))
            key = (n + s_out, qo)
            nxt[key] = nxt[key] + e if key in nxt else e
        E = nxt
    return float(E[(N, 0)][0, 0, 0]) if (N, 0) in E else 0.0


def zipup(x: BMps, mpo: Mpo, m_zip: int, zero_tol: float = tt.ZERO_TOL, per_cut: list | None = None):
    """H x site by site with intermediate rank m_zip.  For m_zip > 0, x is first made
    right-orthogonal.  The carry C_{k-1}[(n, q)] (new bond, operator bond, bond of x) is
    contracted with x_k and W_k (``_site_products``); for every new sector n' the panel
    P = [T2[(n', 0, .)]; T2[(n'-1, 1, .)]] (rows: the new left bond of the U and the O
    block, columns: all (q', b', c')) is factorised, P = U S V^T; across the sectors the
    m_zip largest singular values above the numerical-zero level are kept (``tt.select``
    with tolerance 0; m_zip <= 0: all of them); U[:, :s] gives the new blocks and
    U[:, :s]^T P the next carry.  The last site keeps the panel itself.

    Returns (y, disc2, bound): y equals Q Q^T H x for the orthonormal left basis Q of its
    first L-1 cores; disc2 is the sum of the squared singular values dropped because of
    m_zip (in the panels' own metric), bound whether any was.  per_cut (a list) receives
    the dropped weight of every site 1..L-1."""
    L, N = x.L, x.N
    if m_zip > 0:
        x = right_orthogonalize(x)
    zcap = m_zip if m_zip > 0 else 1 << 60
    rho = empty_rho(L, N)
    blk = [None] + [dict() for _ in range(L)]
    C = {(0, 0): np.ones((1, 1, 1))}
    disc2, bound = 0.0, False
    for k in range(1, L + 1):
        m = k - 1
        T2 = _site_products(mpo, m, C, x, k)
        panels, rows, colq = {}, {}, {}
        for n2 in sectors(L, N, k):
            qcols = []
            for qo in range(-2, 3):
                nx = n2 - qo
                if not _valid(L, N, k, nx):
                    continue
                wq = mpo.wq(k, qo)
                if wq == 0 or x.rho[k][nx] == 0:
                    continue
                qcols.append((qo, wq, x.rho[k][nx]))
            parts, rr = [], []
            for s_out in (0, 1):
                n = n2 - s_out
                if not _valid(L, N, k - 1, n):
                    continue
                r = rho[k - 1][n]
                row = [T2[(n, s_out, qo)].reshape(r, wq * cx) if (n, s_out, qo) in T2 else np.zeros((r, wq * cx))
                       for qo, wq, cx in qcols]
                parts.append(np.hstack(row) if row else np.zeros((r, 0)))
                rr.append((n, s_out, r))
            panels[n2] = np.vstack(parts) if parts else np.zeros((0, 0))
            rows[n2], colq[n2] = rr, qcols
        if k == L:
            P = panels[N]
            off = 0
            for (n, s_out, r) in rows[N]:
                blk[L][(n, s_out)] = P[off:off + r, :].reshape(r, 1) if P.size else np.zeros((r, 1))
                off += r
            for n in sectors(L, N, L - 1):
                for s in (0, 1):
                    if _valid(L, N, L, n + s) and (n, s) not in blk[L]:
                        blk[L][(n, s)] = np.zeros((rho[L - 1][n], 1))
            break
        svd, sv = {}, {}
        for n2, P in panels.items():
            if P.size == 0:
                svd[n2] = (np.zeros((P.shape[0], 0)), np.zeros(0), np.zeros((0, P.shape[1])))
                sv[n2] = np.zeros(0)
                continue
            svd[n2] = _svd(P)
            sv[n2] = svd[n2][1]
        kept, _, _ = tt.select(sv, 0.0, zcap, zero_tol)
        smax = max([s[0] for s in sv.values() if s.size] + [0.0])
        site2 = 0.0
        for n2, s in sv.items():
            dropped = s[kept[n2]:]
            dropped = dropped[dropped > zero_tol * smax]
            if dropped.size:
                site2 += float(np.sum(dropped ** 2))
                bound = True
        disc2 += site2
        if per_cut is not None:
            per_cut.append(site2)
        Cn = {}
        for n2 in sectors(L, N, k):
            U, S, Vt = svd[n2]
            s = kept[n2]
            rho[k][n2] = s
            off = 0
            for (n, s_out, r) in rows[n2]:
                blk[k][(n, s_out)] = U[off:off + r, :s].copy()
                off += r
            carry = U[:, :s].T @ panels[n2] if s else np.zeros((0, panels[n2].shape[1]))
            off = 0
            for qo, wq, cx in colq[n2]:
                Cn[(n2, qo)] = carry[:, off:off + wq * cx].reshape(s, wq, cx)
                off += wq * cx
        # blocks of site k whose right sector has no panel (zero rows) stay empty
        for n in sectors(L, N, k - 1):
            for so in (0, 1):
                if _valid(L, N, k, n + so) and (n, so) not in blk[k]:
                    blk[k][(n, so)] = np.zeros((rho[k - 1][n], rho[k][n + so]))
        C = Cn
    return BMps(L, N, rho, blk), disc2, bound


def apply_h(x: BMps, mpo: Mpo, eps: float, cap: int, m_zip: int, mode: str = "sequential"):
    """trunc(H x; eps, cap) with the zip-up of intermediate rank m_zip.  Returns
    (y, cap_bound, disc2); cap_bound is also set when m_zip dropped a singular value.
    With the simultaneous truncation and m_zip > 0 the panels' numerical-zero level is
    that of the simultaneous truncation (singular values from Gram matrices)."""
    zt = tt.ZERO_TOL_PARALLEL if (mode == "parallel" and m_zip > 0) else tt.ZERO_TOL
    z, disc2, zb = zipup(x, mpo, m_zip, zt)
    y, cb = trunc(z, eps, cap, mode)
    return y, cb or zb, disc2


# ---------------------------------------------------------------- preconditioner


def scaled_terms(pre: precond.Preconditioner, x: BMps):
    """The terms s_m = alpha_m prod_i diag(1, exp(-beta_m theta_i)) x of S x
    (Section 4.3): the O blocks of site i scaled by exp(-beta_m theta_i), alpha_m on
    site 1."""
    out = []
    for a, b in zip(pre.alpha, pre.beta):
        y = x.copy()
        for k in range(1, x.L + 1):
            for (n, s) in y.blk[k]:
                f = math.exp(-b * pre.th[k - 1]) if s == 1 else 1.0
                if k == 1:
                    f *= a
                y.blk[k][(n, s)] = y.blk[k][(n, s)] * f
        out.append(y)
    return out


def apply_s(pre: precond.Preconditioner, x: BMps, eta: float, cap: int, mode: str = "sequential"):
    """S x by the sorted sequential truncated sum (Lemma truncr; as
    ``precond.apply_sorted``): terms by norm ascending (ties: lower m first), the
    leading ones with sum of norms <= eta/3 dropped, y <- trunc_{eps_j}(y + s_j) with
    eps_j = eta ||s_j|| / (3 sum of the kept norms), finally trunc_{eta/3}(y).
    Returns (y, cap_bound)."""
    terms = scaled_terms(pre, x)
    norms = [norm(t) for t in terms]
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
    y, cap_bound = None, False
    for m in rest:
        eps_j = eta * norms[m] / (3.0 * total) if total > 0 else 0.0
        z = terms[m] if y is None else lincomb(1.0, y, 1.0, terms[m])
        y, cb = trunc(z, eps_j, cap, mode)
        cap_bound |= cb
    if y is None:
        return scale(x, 0.0), cap_bound
    y, cb = trunc(y, eta / 3.0, cap, mode)
    return y, cap_bound or cb


# ---------------------------------------------------------------- Algorithm 2


def run(h, v, N, gamma, prm, m_zip=0, psi0: BMps | None = None, mpo: Mpo | None = None, callback=None):
    """Algorithm 2 on block-sparse MPS: the steps, tolerances and records of
    ``pinvit.run`` (see its docstring), with H applied by ``apply_h`` at intermediate rank
    m_zip and every norm an exact transfer sweep.  Returns (psi, hist, pre)."""
    L = h.shape[0]
    pre = precond.Preconditioner(h, v, N, gamma, prm.c0, prm.c_lower, prm.c_upper)
    mode = prm.truncation
    if mpo is None:
        mpo = build_mpo(h, v, gamma / N)
    eps_num = prm.eps_num if prm.eps_num is not None else 0.5 * (1.0 - prm.c)
    zeta = eps_num / (1.0 + prm.c)
    eta = math.inf
    from .pinvit import initial_determinant
    psi = determinant(L, N, initial_determinant(h, N)) if psi0 is None else psi0.copy()
    hist = []
    s_prev = s_prev2 = None
    for it in range(prm.max_iter):
        psi = scale(psi, 1.0 / norm(psi))
        lam = expect(psi, psi, mpo)
        if s_prev is None:
            y0, _, _ = apply_h(psi, mpo, 0.0, prm.cap, m_zip, mode)
            r0, _ = trunc(lincomb(1.0, y0, -lam, psi), 0.0, prm.cap, mode)
            est = pre.s_max * norm(r0)
        elif s_prev2 is None or s_prev2 <= 0.0:
            est = s_prev
        else:
            est = s_prev * min(1.0, s_prev / s_prev2)
        eta = min(2.0 * eta, 0.8 * zeta * est)
        retries = 0
        while True:
            e12 = eta / (3.0 * pre.s_max)
            y, cb1, disc2 = apply_h(psi, mpo, e12, prm.cap, m_zip, mode)
            r, cb2 = trunc(lincomb(1.0, y, -lam, psi), e12, prm.cap, mode)
            s, cb3 = apply_s(pre, r, eta / 3.0, prm.cap, mode)
            cap_bound = cb1 or cb2 or cb3
            ns = norm(s)
            if ns >= (1.0 + 1.0 / zeta) * eta or cap_bound or retries >= prm.max_retries:
                break
            eta *= 0.8
            retries += 1
        p, cb4 = apply_s(pre, s, pre.s_max * eta / 3.0, prm.cap, mode)
        nr = norm(r)
        rho = (ns + eta) / (math.sqrt(1.0 - prm.c) * math.sqrt(lam))
        bound = bounds.eigvec_error_bound(rho, prm.delta)
        rec = dict(it=it, lam=lam, E=lam - gamma, rho=rho, bound=bound, r_norm=nr, s_norm=ns, eta=eta,
                   retries=retries, cap_bound=bool(cap_bound or cb4), zip_disc=math.sqrt(disc2),
                   zip_bound=disc2 > 0.0, max_rank=psi.max_rank())
        # with a binding m_zip the residual is not within eta of the true one: the bound is
        # not certified and the run does not stop on it
        if bound <= prm.tau and not disc2 > 0.0:
            rec["stop"] = True
            hist.append(rec)
            break
        npn = norm(p)
        if npn == 0.0:
            rec["stop"] = True
            rec["direction_vanished"] = True
            hist.append(rec)
            break
        z2 = scale(p, 1.0 / npn)
        h12 = expect(psi, z2, mpo)
        h22 = expect(z2, z2, mpo)
        o12 = dot(psi, z2)
        hm = np.array([[lam, h12], [h12, h22]])
        mm = np.array([[1.0, o12], [o12, 1.0]])
        lam_s, vv = bounds.ritz2(hm, mm)
        q = math.sqrt(lam_s / (lam_s + prm.t_eig * (lam - lam_s)))
        da = bounds.delta_a(rho, q)
        eta_in = da * math.sqrt(lam_s) / math.sqrt(1.0 + prm.c)
        eta_psi = eta_in * pre.s_min
        psi, cb5 = trunc(lincomb(vv[0], psi, vv[1], z2), eta_psi, prm.cap, mode)
        rec.update(lam_star=lam_s, eta_psi=eta_psi, cap_bound=rec["cap_bound"] or bool(cb5),
                   max_rank=psi.max_rank(), rho_tab=psi.rho.copy())
        hist.append(rec)
        if callback is not None:
            callback(rec, psi)
        s_prev2, s_prev = s_prev, ns
    return psi, hist, pre
