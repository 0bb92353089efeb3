"""Seeded random block-sparse MPS in the export layout (test and benchmark inputs).

Block tables: at cut k the sectors are n in {max(0,N-L+k) .. min(N,k)}; the full
rank of sector n is min(C(k,n), C(L-k,N-n)).  ``rho_table(L, N, cap)`` spreads a
total rank ``cap`` over the sectors in proportion to C(k,n) C(L-k,N-n), never above
the full rank and at least 1, and uses the full ranks when they sum to <= cap.
Cores are i.i.d. N(0, 1/rows) in the layout described in the library header.
"""
from __future__ import annotations

import math

import numpy as np


def sectors(L: int, N: int, k: int):
    return list(range(max(0, N - L + k), min(N, k) + 1))


def rho_table(L: int, N: int, cap: int) -> np.ndarray:
    rho = np.zeros((L + 1, N + 1), dtype=np.int32)
    for k in range(L + 1):
        secs = sectors(L, N, k)
        full = {n: min(math.comb(k, n), math.comb(L - k, N - n)) for n in secs}
        if sum(full.values()) <= cap:
            for n in secs:
                rho[k, n] = full[n]
            continue
        w = {n: math.comb(k, n) * math.comb(L - k, N - n) for n in secs}
        tot = sum(w.values())
        for n in secs:
            rho[k, n] = min(full[n], max(1, int(round(cap * w[n] / tot))))
    return rho


def layout(L: int, N: int, rho):
    """[(k, n, kind, rows, cols)] in export order (kind 0 = unoccupied, 1 = occupied)."""
    out = []
    for k in range(1, L + 1):
        right = set(sectors(L, N, k))
        for n in sectors(L, N, k - 1):
            if n in right:
                out.append((k, n, 0, int(rho[k - 1][n]), int(rho[k][n])))
            if n + 1 in right:
                out.append((k, n, 1, int(rho[k - 1][n]), int(rho[k][n + 1])))
    return out


def random_block_mps(L: int, N: int, rho, seed: int, isometric: bool = False) -> np.ndarray:
    """Random cores in export layout.  isometric=True draws, for every site k and right
    sector n, the stacked blocks [U(k, n); O(k, n - 1)] as a random matrix with orthonormal
    columns (Q of a Gaussian matrix; a scaled Gaussian when it has fewer rows than
    columns), which gives states whose left parts are orthonormal: a well-conditioned gauge
    like that of truncated iterates, without which Gram-based singular values lose accuracy
    in proportion to the gauge's condition."""
    rng = np.random.default_rng(seed)
    if not isometric:
        parts = []
        for _, _, _, r, c in layout(L, N, rho):
            parts.append(rng.standard_normal(r * c) / math.sqrt(max(r, 1)))
        return np.concatenate(parts) if parts else np.zeros(0)
    blocks = {}
    for k in range(1, L + 1):
        left = set(sectors(L, N, k - 1))
        for n in sectors(L, N, k):
            parts = [(n, 0)] if n in left else []
            if n - 1 in left:
                parts.append((n - 1, 1))
            rows = [int(rho[k - 1][m]) for m, _ in parts]
            R, c = sum(rows), int(rho[k][n])
            g = rng.standard_normal((R, c))
            if R >= c and c > 0:
                q, _ = np.linalg.qr(g)
            else:
                q = g / math.sqrt(max(R, 1))
            r0 = 0
            for (m, kind), r in zip(parts, rows):
                blocks[(k, m, kind)] = q[r0:r0 + r, :]
                r0 += r
    out = [blocks[(k, n, kind)].reshape(-1, order="F") for k, n, kind, _, _ in layout(L, N, rho)]
    return np.concatenate(out) if out else np.zeros(0)
