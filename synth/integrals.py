"""Random integrals (h, v) with the symmetries of a real orbital basis, and the shift.

Conventions (these are data conventions, fixed once for the whole repository):

* ``h`` is an L x L symmetric array; the one-body part is sum_ij h[i,j] a_i^* a_j.
* ``v`` is an L^4 array whose entry v[i,j,k,l] multiplies a_i^* a_j^* a_k a_l
  directly (the factor one half of the paper's definition of v is already inside).
  It is produced from a chemist-notation tensor g with the 8-fold real symmetry,
  g[p,q,r,s] = (pq|rs), by v[i,j,k,l] = g[i,l,j,k] / 2, which is the paper's
  v_ijkl = 1/2 * integral phi_i(x1) phi_j(x2) V phi_k(x2) phi_l(x1)
  (Section 1.1, definition of t_ij and v_ijkl).
* Orbital i of the paper is index i-1 here.

Recipes (all draws from numpy's PCG64 ``default_rng(seed)``, in the order listed):

``dense`` (the small validation case):
    h upper triangle (incl. diagonal) i.i.d. N(0, 1), mirrored;
    g canonical index classes i.i.d. N(0, 0.1^2), copied to all 8 images.
``decayed`` (the scaling workloads):
    z upper triangle i.i.d. N(0,1), mirrored; eps_i i.i.d. U(-2, 1), sorted ascending;
    h_ij = z_ij exp(-|i-j|/4) + delta_ij eps_i;
    g = (8-fold symmetric N(0, 0.1^2) draw) * exp(-(|p-q| + |r-s|)/4).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def _sym_matrix(rng: np.random.Generator, L: int, scale: float = 1.0) -> np.ndarray:
    iu = np.triu_indices(L)
    a = np.zeros((L, L))
    a[iu] = rng.standard_normal(len(iu[0])) * scale
    return a + np.triu(a, 1).T


def sym8(rng: np.random.Generator, L: int, scale: float) -> np.ndarray:
    """A 4-index array with g[p,q,r,s] = g[q,p,r,s] = g[p,q,s,r] = g[r,s,p,q].

    One i.i.d. N(0, scale^2) value is drawn per canonical index class (the
    lexicographically smallest of the 8 images), classes taken in ascending
    order of their flat index, and copied to every image.
    """
    idx = np.indices((L, L, L, L)).reshape(4, -1)
    p, q, r, s = idx

    def flat(a, b, c, d):
        return ((a * L + b) * L + c) * L + d

    images = np.stack([
        flat(p, q, r, s), flat(q, p, r, s), flat(p, q, s, r), flat(q, p, s, r),
        flat(r, s, p, q), flat(s, r, p, q), flat(r, s, q, p), flat(s, r, q, p),
    ])
    canon = images.min(axis=0)
    classes, inverse = np.unique(canon, return_inverse=True)
    vals = rng.standard_normal(len(classes)) * scale
    return vals[inverse].reshape(L, L, L, L)


def v_from_chemist(g: np.ndarray) -> np.ndarray:
    """v[i,j,k,l] = g[i,l,j,k] / 2 (see the module docstring)."""
    return 0.5 * np.ascontiguousarray(np.transpose(g, (0, 2, 3, 1)))


def random_dense(L: int, seed: int):
    rng = np.random.default_rng(seed)
    h = _sym_matrix(rng, L)
    g = sym8(rng, L, 0.1)
    return h, v_from_chemist(g)


def random_decayed(L: int, seed: int):
    rng = np.random.default_rng(seed)
    z = _sym_matrix(rng, L)
    eps = np.sort(rng.uniform(-2.0, 1.0, size=L))
    i = np.arange(L)
    dist = np.abs(i[:, None] - i[None, :])
    h = z * np.exp(-dist / 4.0) + np.diag(eps)
    g = sym8(rng, L, 0.1)
    g = g * np.exp(-(dist[:, :, None, None] + dist[None, None, :, :]) / 4.0)
    return h, v_from_chemist(g)


def shift_lower_bound(h: np.ndarray, v: np.ndarray, N: int) -> float:
    """Shift gamma = 1 - E_lb with E_lb a rigorous lower bound of the N-particle energy.

    E_lb = (sum of the N smallest eigenvalues of h) + C(N,2) * lambda_min(V_2), where
    V_2 is the two-body operator on the two-particle space, basis a_p^* a_q^*|0>,
    p < q, whose matrix is -(v_ijpq - v_jipq - v_ijqp + v_jiqp) for pairs (i<j),(p<q).
    Then H + gamma has all N-particle eigenvalues >= 1.
    """
    L = h.shape[0]
    e1 = np.sort(np.linalg.eigvalsh(h))[:N].sum()
    if N < 2:
        return float(1.0 - e1)
    iu, ju = np.triu_indices(L, 1)
    w = v - v.transpose(1, 0, 2, 3) - v.transpose(0, 1, 3, 2) + v.transpose(1, 0, 3, 2)
    v2 = -w[iu, ju][:, iu, ju]
    v2 = 0.5 * (v2 + v2.T)
    lmin = np.linalg.eigvalsh(v2)[0]
    return float(1.0 - (e1 + math.comb(N, 2) * lmin))


@dataclasses.dataclass
class Problem:
    kind: str
    L: int
    N: int
    seed: int
    h: np.ndarray
    v: np.ndarray
    gamma: float


def make_problem(kind: str, L: int, N: int, seed: int = 0) -> Problem:
    if kind == "dense":
        h, v = random_dense(L, seed)
    elif kind == "decayed":
        h, v = random_decayed(L, seed)
    else:
        raise ValueError(f"unknown integral kind {kind!r}")
    return Problem(kind, L, N, seed, h, v, shift_lower_bound(h, v, N))
