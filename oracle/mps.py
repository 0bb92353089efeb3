"""Dense vector of a block-sparse MPS given in the library's export layout (oracle).

Layout (one float64 array): sites k = 1..L in order; inside a site, left sectors
n in K_{k-1} ascending; for each, the unoccupied block U_{k,n} (rho_{k-1,n} x rho_{k,n},
present when n in K_k) then the occupied block O_{k,n} (rho_{k-1,n} x rho_{k,n+1},
present when n+1 in K_k); each block column-major (Section 2.3, eq. blockstructure).
``rho`` is an (L+1) x (N+1) integer table, zero outside K_k.

The dense vector follows eq. mps: x_alpha = X_1^{alpha_1} ... X_L^{alpha_L}, where
X_k^{0} holds the U blocks on the block diagonal and X_k^{1} the O blocks just above it.
"""
from __future__ import annotations

import numpy as np

from .tt import sectors


def block_shapes(L: int, N: int, rho):
    """[(k, n, kind, rows, cols)] in export order, kind 0 = U, 1 = O."""
    out = []
    for k in range(1, L + 1):
        right = set(sectors(L, N, k))
        for n in sectors(L, N, k - 1):
            if n in right:
                out.append((k, n, 0, int(rho[k - 1][n]), int(rho[k][n])))
            if n + 1 in right:
                out.append((k, n, 1, int(rho[k - 1][n]), int(rho[k][n + 1])))
    return out


def size(L, N, rho) -> int:
    return sum(r * c for _, _, _, r, c in block_shapes(L, N, rho))


def unpack(L, N, rho, data):
    """{(k, n, kind): 2-D block}."""
    out = {}
    off = 0
    for k, n, kind, r, c in block_shapes(L, N, rho):
        out[(k, n, kind)] = np.asarray(data[off:off + r * c], dtype=np.float64).reshape(c, r).T
        off += r * c
    if off != len(data):
        raise ValueError(f"data length {len(data)} != layout size {off}")
    return out


def to_dense(L, N, rho, data) -> np.ndarray:
    blk = unpack(L, N, rho, data)
    # phi[n] = (configs over the first k orbitals with n particles, matrix configs x rho)
    phi = {0: (np.array([0], dtype=np.int64), np.ones((1, 1)))}
    for k in range(1, L + 1):
        new = {}
        for n2 in sectors(L, N, k):
            cfgs, mats = [], []
            if (k, n2, 0) in blk and n2 in phi:
                c, m = phi[n2]
                cfgs.append(c)
                mats.append(m @ blk[(k, n2, 0)])
            if (k, n2 - 1, 1) in blk and n2 - 1 in phi:
                c, m = phi[n2 - 1]
                cfgs.append(c | (1 << (k - 1)))
                mats.append(m @ blk[(k, n2 - 1, 1)])
            if cfgs:
                new[n2] = (np.concatenate(cfgs), np.vstack(mats))
        phi = new
    x = np.zeros(1 << L)
    cfg, mat = phi[N]
    x[cfg] = mat[:, 0]
    return x


def amplitude(L, N, rho, data, config: int) -> float:
    """x_alpha for one occupation pattern (bit i-1 = orbital i), by the matrix product."""
    blk = unpack(L, N, rho, data)
    vec = np.ones((1, 1))
    n = 0
    for k in range(1, L + 1):
        occ = config >> (k - 1) & 1
        key = (k, n, occ)
        if key not in blk:
            return 0.0
        vec = vec @ blk[key]
        n += occ
    return float(vec[0, 0]) if n == N else 0.0
