"""Occupation-number space, Jordan-Wigner operators and the Hamiltonian (oracle).

Basis: the index of a vector of length 2^L is sum_i alpha_i 2^(i-1), alpha_i the
occupation of orbital i (Section 1.1: Slater determinants <-> binary alpha).

a_i = S x ... x S x A x I x ... x I with S = diag(1,-1), A = [[0,1],[0,0]]
(Section 1.1, definition of the annihilation operator and its elementary
components).  Hence (a_i x)[beta] = (-1)^(#occupied orbitals < i in beta) x[beta + e_i]
for beta with alpha_i = 0, and 0 otherwise.

Pins: ``kron_ops`` is the literal Kronecker-product definition; the tests check the
bit-string operators against it and the anticommutation relations (eq. anticomm).
"""
from __future__ import annotations

import functools
import math

import numpy as np

_S = np.diag([1.0, -1.0])
_A = np.array([[0.0, 1.0], [0.0, 0.0]])
_I = np.eye(2)


def kron_ops(L: int):
    """Dense 2^L x 2^L matrices a_1..a_L from the Kronecker definition.

    np.kron puts its first factor (orbital 1) in the most significant position; the
    result is permuted to this module's ordering (orbital 1 = least significant bit).
    Use only for L <= 8.
    """
    dim = 1 << L
    perm = np.zeros(dim, dtype=np.int64)
    for idx in range(dim):
        # kron index has orbital 1 as the highest bit: reverse the bits
        rev = 0
        for b in range(L):
            if idx >> b & 1:
                rev |= 1 << (L - 1 - b)
        perm[rev] = idx
    ops = []
    for i in range(L):
        m = np.ones((1, 1))
        for k in range(L):
            m = np.kron(m, _S if k < i else (_A if k == i else _I))
        # m is indexed in kron order; perm maps kron index -> bit index
        out = np.zeros_like(m)
        out[np.ix_(perm, perm)] = m
        ops.append(out)
    return ops


@functools.lru_cache(maxsize=None)
def _annihilation_map(L: int, i: int):
    idx = np.arange(1 << L, dtype=np.int64)
    dst = idx[(idx >> i & 1) == 0]
    src = dst | (1 << i)
    below = dst & ((1 << i) - 1)
    parity = np.array([bin(int(b)).count("1") & 1 for b in below], dtype=np.int64)
    sign = 1.0 - 2.0 * parity
    return dst, src, sign


def annihilate(x: np.ndarray, i: int) -> np.ndarray:
    """a_i x (i zero-based) for x of shape (2^L, ...)."""
    L = x.shape[0].bit_length() - 1
    dst, src, sign = _annihilation_map(L, i)
    out = np.zeros_like(x)
    out[dst] = (sign.reshape((-1,) + (1,) * (x.ndim - 1))) * x[src]
    return out


def create(x: np.ndarray, i: int) -> np.ndarray:
    """a_i^* x: the transpose of annihilate (a_i is real)."""
    L = x.shape[0].bit_length() - 1
    dst, src, sign = _annihilation_map(L, i)
    out = np.zeros_like(x)
    out[src] = (sign.reshape((-1,) + (1,) * (x.ndim - 1))) * x[dst]
    return out


def apply_h(h: np.ndarray, v: np.ndarray, x: np.ndarray, gamma: float = 0.0) -> np.ndarray:
    """(H + gamma I) x with H = sum h_ij a_i^* a_j + sum v_ijkl a_i^* a_j^* a_k a_l.

    Section 1.1, eq. hamil, applied term by term: Y_kl = a_k a_l x for all (k,l), then
    Z_ij = sum_kl v_ijkl Y_kl (one matrix product), then sum_ij a_i^* a_j^* Z_ij.
    """
    L = h.shape[0]
    out = gamma * x
    ax = [annihilate(x, j) for j in range(L)]
    for i in range(L):
        acc = np.zeros_like(x)
        for j in range(L):
            if h[i, j] != 0.0:
                acc += h[i, j] * ax[j]
        out = out + create(acc, i)
    y = np.stack([annihilate(ax[l], k) for k in range(L) for l in range(L)])
    z = (v.reshape(L * L, L * L) @ y.reshape(L * L, -1)).reshape(y.shape)
    for i in range(L):
        acc = np.zeros_like(x)
        for j in range(L):
            acc += create(z[i * L + j], j)
        out = out + create(acc, i)
    return out


def number_op(x: np.ndarray) -> np.ndarray:
    """P x = sum_i a_i^* a_i x (particle-number operator, Section 1.1)."""
    L = x.shape[0].bit_length() - 1
    out = np.zeros_like(x)
    for i in range(L):
        out += create(annihilate(x, i), i)
    return out


def sector_basis(L: int, N: int) -> np.ndarray:
    """Indices of the N-particle states in ascending order (dimension C(L, N))."""
    idx = np.arange(1 << L, dtype=np.int64)
    pc = np.array([bin(int(b)).count("1") for b in idx])
    return idx[pc == N]


def sector_hamiltonian(h, v, N, gamma=0.0, chunk=64):
    """Dense matrix of H + gamma on the N-particle sector (eq. Hevp), by applying H
    to unit vectors.  Exact diagonalisation for small L."""
    L = h.shape[0]
    basis = sector_basis(L, N)
    d = len(basis)
    H = np.zeros((d, d))
    for c0 in range(0, d, chunk):
        cols = basis[c0:c0 + chunk]
        X = np.zeros((1 << L, len(cols)))
        X[cols, np.arange(len(cols))] = 1.0
        Y = apply_h(h, v, X, gamma)
        H[:, c0:c0 + len(cols)] = Y[basis]
    return H


def lowest_eigs(h, v, N, gamma=0.0, k=2):
    """The k lowest eigenvalues of H + gamma on the N-particle sector.

    Dense eigh for sector dimension <= 4000, else Lanczos (scipy eigsh) with the
    matrix-free apply_h."""
    L = h.shape[0]
    basis = sector_basis(L, N)
    d = len(basis)
    if d <= 4000:
        w = np.linalg.eigvalsh(sector_hamiltonian(h, v, N, gamma))
        return w[:k]
    from scipy.sparse.linalg import LinearOperator, eigsh

    def mv(y):
        x = np.zeros(1 << L)
        x[basis] = y.ravel()
        return apply_h(h, v, x, gamma)[basis]

    op = LinearOperator((d, d), matvec=mv, dtype=np.float64)
    w = eigsh(op, k=k, which="SA", tol=1e-13, return_eigenvectors=False)
    return np.sort(w)


def determinant(L: int, occupied) -> np.ndarray:
    """Unit vector of the Slater determinant with the given zero-based orbitals."""
    x = np.zeros(1 << L)
    x[sum(1 << i for i in occupied)] = 1.0
    return x


def comb(n, k):
    return math.comb(n, k) if 0 <= k <= n else 0
