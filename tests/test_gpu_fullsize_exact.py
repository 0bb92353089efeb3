"""Exact checks at the benchmark's size (L = 48, N = 24, the full MPO with bond 1226):
the sandwich <a|H_gamma|b> between determinant MPS and the H application to a
determinant, against the matrix elements of the Slater-Condon selection evaluated one by
one on bit strings (oracle/slater.py): diagonal elements, single and double excitations,
and zeros beyond them."""
import numpy as np
import pytest

from oracle import slater
from synth import make_problem

pytestmark = pytest.mark.gpu

native = pytest.importorskip("paper_2604_16118_amd.native")

L, N = 48, 24


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = native.Context(0)
    p = make_problem("decayed", L, N, 0)
    ctx.set_hamiltonian(p.h, p.v, N, p.gamma)
    ctx.set_truncation(0)
    rng = np.random.default_rng(48)
    b0 = sum(1 << i for i in np.argsort(np.diag(p.h), kind="stable")[:N])  # the start determinant
    singles = slater.single_excitations(b0, L)
    doubles = slater.double_excitations(b0, L)
    pick = lambda xs, k: [xs[int(i)] for i in rng.choice(len(xs), k, replace=False)]
    triples = []
    for d in pick(doubles, 10):
        occ = [i for i in range(L) if d >> i & 1 and b0 >> i & 1]
        emp = [i for i in range(L) if not d >> i & 1 and not b0 >> i & 1]
        triples.append(d ^ (1 << occ[int(rng.integers(len(occ)))]) ^ (1 << emp[int(rng.integers(len(emp)))]))
    # a second reference determinant far from the first (random N orbitals)
    b1 = sum(1 << int(i) for i in rng.choice(L, N, replace=False))
    targets = [b0] + pick(singles, 40) + pick(doubles, 60) + triples
    handles = {}

    def det(mask):
        if mask not in handles:
            handles[mask] = ctx.mps_determinant([i for i in range(L) if mask >> i & 1])
        return handles[mask]

    yield ctx, p, b0, b1, targets, det
    for h in handles.values():
        ctx.mps_free(h)
    ctx.close()


def test_sandwich_between_determinants_equals_slater_condon(setup):
    ctx, p, b0, b1, targets, det = setup
    scale = np.abs(p.h).max() * N
    for b in (b0, b1):
        for a in targets + [b1]:
            want = slater.element(p.h, p.v, p.gamma, a, b)
            got = ctx.expect_h(det(a), det(b))
            assert got == pytest.approx(want, abs=1e-12 * scale), (bin(a ^ b).count("1") // 2, got, want)


def test_h_applied_to_a_determinant_has_the_slater_condon_amplitudes(setup):
    """H_gamma |b> by the exact zip-up (m_zip <= 0) and a truncation with eps = 0: its
    overlaps with determinants a are <a|H_gamma|b>."""
    ctx, p, b0, b1, targets, det = setup
    y, cb = ctx.apply_h(det(b0), 0.0, 10 ** 6, 0)
    assert not cb
    norm_hy = np.sqrt(ctx.dot(y, y))
    for a in targets:
        want = slater.element(p.h, p.v, p.gamma, a, b0)
        assert ctx.dot(det(a), y) == pytest.approx(want, abs=1e-11 * norm_hy)
    # the norm: sum of the squares of all amplitudes, each a Slater-Condon element
    allw = [slater.element(p.h, p.v, p.gamma, a, b0)
            for a in [b0] + slater.single_excitations(b0, L) + slater.double_excitations(b0, L)]
    assert norm_hy ** 2 == pytest.approx(float(np.sum(np.square(allw))), rel=1e-11)
    ctx.mps_free(y)
