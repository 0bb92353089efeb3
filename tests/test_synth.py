"""Seeded input generators: block tables and random block-sparse MPS."""
import numpy as np

from oracle import mps as omps
from synth import random_block_mps, rho_table
from synth.mps import layout


def test_rho_table_full_ranks_and_cap():
    L, N = 10, 5
    full = rho_table(L, N, 10 ** 6)
    assert full[5, 2] == 10 and full[5, 3] == 10  # min(C(5,n), C(5,5-n))
    capped = rho_table(L, N, 12)
    assert capped[5].sum() <= 12 + len(range(0, 6))  # rounding and the floor of one
    assert np.all(capped <= full)


def test_isometric_mps_has_unit_norm_and_layout_size():
    L, N = 12, 6
    rho = rho_table(L, N, 40)
    data = random_block_mps(L, N, rho, 3, isometric=True)
    assert data.size == sum(r * c for *_, r, c in layout(L, N, rho))
    x = omps.to_dense(L, N, rho, data)
    assert abs(np.linalg.norm(x) - 1.0) <= 1e-12
    # deterministic in the seed
    assert np.array_equal(data, random_block_mps(L, N, rho, 3, isometric=True))
