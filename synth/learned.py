"""Seeded inputs of the learned preconditioner correction: initial network parameters and
the sampled determinants of its training set (occupation bit masks).  Random numbers
only; the network, its loss and the preconditioner are computed elsewhere."""
from __future__ import annotations

import numpy as np

N_FEAT = 6
WIDTH = 256
# flat float32 parameter vector: W1 (WIDTH x N_FEAT, row-major), b1, W2 (WIDTH x WIDTH),
# b2, W3 (WIDTH), b3
N_PARAMS = WIDTH * N_FEAT + WIDTH + WIDTH * WIDTH + WIDTH + WIDTH + 1


def init_params(seed: int = 0, out_scale: float = 0.1) -> np.ndarray:
    """Gaussian weights with variance 1/fan_in (the output layer scaled by out_scale),
    zero biases."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((WIDTH, N_FEAT)) / np.sqrt(N_FEAT)
    w2 = rng.standard_normal((WIDTH, WIDTH)) / np.sqrt(WIDTH)
    w3 = out_scale * rng.standard_normal(WIDTH) / np.sqrt(WIDTH)
    p = np.concatenate([w1.ravel(), np.zeros(WIDTH), w2.ravel(), np.zeros(WIDTH), w3, np.zeros(1)])
    return p.astype(np.float32)


def sample_determinants(L: int, N: int, count: int, seed: int = 0, start=None, max_exc: int = 3) -> np.ndarray:
    """count N-particle occupation masks (uint64, bit i = orbital i): half drawn uniformly,
    half as 1..max_exc random excitations of the start determinant `start` (a list of N
    orbitals; orbitals 0..N-1 when None)."""
    if L > 64:
        raise ValueError("masks hold at most 64 orbitals")
    rng = np.random.default_rng(seed)
    start = list(range(N)) if start is None else list(start)
    out = np.zeros(count, dtype=np.uint64)
    for b in range(count):
        if b % 2 == 0 or N == 0 or N == L:
            occ = rng.choice(L, size=N, replace=False)
        else:
            occ = set(start)
            virt = [a for a in range(L) if a not in occ]
            k = int(rng.integers(1, min(max_exc, N, L - N) + 1))
            for i in rng.choice(sorted(occ), size=k, replace=False):
                occ.discard(int(i))
            for a in rng.choice(virt, size=k, replace=False):
                occ.add(int(a))
            occ = np.array(sorted(occ))
        m = 0
        for i in occ:
            m |= 1 << int(i)
        out[b] = np.uint64(m)
    return out
