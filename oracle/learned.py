"""Learned correction of the preconditioner's diagonal (oracle; test infrastructure only).

An extension, not part of the paper.  The paper's S is built from the diagonal
approximation D = sum_i theta_i n_i of H + gamma (Section 7.1.1, Cor. lrprecond).  Here a
small network corrects theta_i per site i and per number n of particles on the sites
before i (the left sector of the site in the block-sparse MPS), so that each of the M
terms of S stays a product of block-diagonal site factors (rank one per term):

    d(beta) = sum_{i occupied in beta} (theta_i + Delta_{i, n_i(beta)}),
    S_m(beta) = alpha_m exp(-beta_m d(beta)),

with t_min and t_max the extremes of d over the N-particle determinants (a shortest and a
longest path over (site, particles so far)), from which T, h, M+-, alpha_m, beta_m, s_min
and s_max follow as for the plain S.  Delta = delta_max tanh(z) with
delta_max = min_i theta_i / 2, so d stays positive and S positive definite.

Network: per (i, n) the features
    theta_i / tbar, h_ii / tbar, n / N, i / L, <n_i> of the iterate, lambda / (N tbar)
(tbar = mean |theta_i|), two hidden layers of width 256 with tanh, a linear output z.
Parameters are float32; the forward and backward passes use them rounded to bfloat16
(round to nearest even).

Training: Adam on the mean squared misfit between d and the exact diagonal of H + gamma
on sampled determinants,
    loss = mean_b (d(beta_b) - <beta_b|H + gamma|beta_b>)^2 / tbar^2,
    <beta|H + gamma|beta> = gamma + sum_i h_ii n_i + sum_{i != j} (v_ijji - v_ijij) n_i n_j,
so that S approximates (H + gamma)^{-1/2} on the diagonal more closely.  The solve form
(``exact_solve``, ``solve_loss_grad``, at the end) trains instead on exact solves of the
method's own residuals.  Arithmetic here is float64.
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT = 6
WIDTH = 256


def bf16(x) -> np.ndarray:
    """float32 values rounded to bfloat16 (nearest, ties to even), returned as float64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    """(W1, b1, W2, b2, W3, b3) of the flat parameter vector, rounded to bfloat16."""
    q = bf16(p)
    o = 0
    out = []
    for shape in [(WIDTH, N_FEAT), (WIDTH,), (WIDTH, WIDTH), (WIDTH,), (WIDTH,), (1,)]:
        n = int(np.prod(shape))
        out.append(q[o:o + n].reshape(shape))
        o += n
    return out


def densities(x: np.ndarray) -> np.ndarray:
    """<n_i> = sum_beta x_beta^2 [bit i of beta] / sum_beta x_beta^2."""
    L = x.shape[0].bit_length() - 1
    idx = np.arange(x.shape[0], dtype=np.int64)
    w = x * x
    return np.array([w[((idx >> i) & 1) == 1].sum() for i in range(L)]) / w.sum()


def features(th, hdiag, dens, lam, N) -> np.ndarray:
    """(L (N+1)) x 6 features, row i (N+1) + n."""
    L = len(th)
    tbar = float(np.mean(np.abs(th)))
    X = np.zeros((L * (N + 1), N_FEAT))
    for i in range(L):
        for n in range(N + 1):
            X[i * (N + 1) + n] = [th[i] / tbar, hdiag[i] / tbar, n / N, i / L, dens[i], lam / (N * tbar)]
    return X


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    z = h2 @ W3 + b3[0]
    return z, (h1, h2)


def delta_max(th) -> float:
    m = float(np.min(th))
    return 0.5 * m if m > 0 else 0.0


def correction(p, X, dmax, L, N) -> np.ndarray:
    """Delta as an L x (N+1) table."""
    z, _ = forward(p, X)
    return (dmax * np.tanh(z)).reshape(L, N + 1)


def _occ_left(mask: int, L: int):
    """[(i, particles on sites < i)] for the occupied sites of a mask."""
    out, n = [], 0
    for i in range(L):
        if (mask >> i) & 1:
            out.append((i, n))
            n += 1
    return out


def exact_diagonal(h, v, gamma, masks) -> np.ndarray:
    L = h.shape[0]
    out = np.zeros(len(masks))
    for b, m in enumerate(masks):
        occ = [i for i in range(L) if (int(m) >> i) & 1]
        e = gamma + sum(h[i, i] for i in occ)
        for i in occ:
            for j in occ:
                if i != j:
                    e += v[i, j, j, i] - v[i, j, i, j]
        out[b] = e
    return out


def approx_diagonal(th, delta, masks) -> np.ndarray:
    L = len(th)
    return np.array([sum(th[i] + delta[i, n] for i, n in _occ_left(int(m), L)) for m in masks])


def loss_grad(p, X, dmax, th, masks, targets, N):
    """(loss, gradient of the loss with respect to the (bfloat16-rounded) parameters)."""
    L = len(th)
    tbar = float(np.mean(np.abs(th)))
    W1, b1, W2, b2, W3, b3 = unpack(p)
    z, (h1, h2) = forward(p, X)
    tz = np.tanh(z)
    delta = (dmax * tz).reshape(L, N + 1)
    e = approx_diagonal(th, delta, masks) - targets
    B = len(masks)
    loss = float(np.mean(e * e)) / (tbar * tbar)
    G = np.zeros((L, N + 1))
    for b, m in enumerate(masks):
        for i, n in _occ_left(int(m), L):
            G[i, n] += 2.0 * e[b] / (B * tbar * tbar)
    dz = G.ravel() * dmax * (1.0 - tz * tz)
    gW3 = h2.T @ dz
    gb3 = np.array([dz.sum()])
    da2 = np.outer(dz, W3) * (1.0 - h2 * h2)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * (1.0 - h1 * h1)
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    return loss, np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, gb3])


def train(p, X, dmax, th, masks, targets, N, steps, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam from zero moments; returns (float32 parameters, losses before each step and
    after the last)."""
    w = np.asarray(p, dtype=np.float64).copy()
    m = np.zeros_like(w)
    s = np.zeros_like(w)
    losses = []
    for t in range(1, steps + 1):
        loss, g = loss_grad(w, X, dmax, th, masks, targets, N)
        losses.append(loss)
        m = b1 * m + (1 - b1) * g
        s = b2 * s + (1 - b2) * g * g
        w = w - lr * (m / (1 - b1 ** t)) / (np.sqrt(s / (1 - b2 ** t)) + eps)
        w = w.astype(np.float32).astype(np.float64)  # the parameters are float32
    losses.append(loss_grad(w, X, dmax, th, masks, targets, N)[0])
    return w.astype(np.float32), losses


def t_range(th, delta, N):
    """(min, max) of d over the N-particle determinants: dynamic programming over the
    sites with the number of particles placed so far as the state."""
    L = len(th)
    lo = np.full(N + 1, math.inf)
    hi = np.full(N + 1, -math.inf)
    lo[0] = hi[0] = 0.0
    for i in range(L):
        nlo, nhi = lo.copy(), hi.copy()
        for n in range(1, N + 1):
            c = th[i] + delta[i, n - 1]
            nlo[n] = min(lo[n], lo[n - 1] + c)
            nhi[n] = max(hi[n], hi[n - 1] + c)
        lo, hi = nlo, nhi
    return float(lo[N]), float(hi[N])


# ---------------------------------------------------------------- exact-solve targets
#
# The training target of the solve form: the exact solve t = (H + gamma)^{-1} r on the
# N-particle sector of a residual r that the method generates, and the corrected
# diagonal preconditioner's action r / d on the same vector.  Trained on sampled
# determinants b, the misfit
#     loss = sum_b (r_b / d(beta_b) - t_b)^2 / sum_b t_b^2
# asks S^2 (which is close to D^{-1}, alpha_0^2 t_min S(d/t_min)^2 ~ 1/d) to act on the
# method's residuals like the exact inverse of H + gamma.


def exact_solve(h, v, N, gamma, r):
    """t = (H + gamma)^{-1} r on the N-particle sector (dense solve; r a 2^L vector)."""
    from . import fock
    L = h.shape[0]
    basis = fock.sector_basis(L, N)
    H = fock.sector_hamiltonian(h, v, N, gamma)
    t = np.zeros(1 << L)
    t[basis] = np.linalg.solve(H, r[basis])
    return t


def solve_loss_grad(p, X, dmax, th, masks, rvals, tvals, N):
    """(loss, gradient) of the solve misfit above with respect to the (bfloat16-rounded)
    parameters."""
    L = len(th)
    W1, b1, W2, b2, W3, b3 = unpack(p)
    z, (h1, h2) = forward(p, X)
    tz = np.tanh(z)
    delta = (dmax * tz).reshape(L, N + 1)
    d = approx_diagonal(th, delta, masks)
    rv, tv = np.asarray(rvals, float), np.asarray(tvals, float)
    nt = float(np.sum(tv * tv))
    e = rv / d - tv
    loss = float(np.sum(e * e)) / nt
    gd = -2.0 * e * rv / (d * d) / nt   # d loss / d d_b
    G = np.zeros((L, N + 1))
    for b, m in enumerate(masks):
        for i, n in _occ_left(int(m), L):
            G[i, n] += gd[b]
    dz = G.ravel() * dmax * (1.0 - tz * tz)
    gW3 = h2.T @ dz
    gb3 = np.array([dz.sum()])
    da2 = np.outer(dz, W3) * (1.0 - h2 * h2)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * (1.0 - h1 * h1)
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    return loss, np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, gb3])
