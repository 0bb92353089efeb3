"""Matrix elements of H between Slater determinants (oracle).  TEST INFRASTRUCTURE ONLY.

Only the test-suite may use this module; the GPU library shares no code with it.

A determinant is a bit mask: bit i set = orbital i+1 occupied (Section 1.1: Slater
determinants <-> binary alpha).  <a| H + gamma |b> for H = sum h_ij a_i^* a_j +
sum v_ijkl a_i^* a_j^* a_k a_l (eq. hamil) is computed by applying the terms of H to b
literally: each operator acts on the bit string with the Jordan-Wigner sign
(-1)^(number of occupied orbitals below the one it acts on) (eq. anniloperator), the
rightmost operator first.  Only terms that can map b to a are visited (the selection
rule of the Slater-Condon rules: a product of two creators and two annihilators changes
at most two occupations), which keeps the cost independent of 2^L, so the elements are
available at L = 48 and beyond.
"""
from __future__ import annotations

import itertools


def _bits(mask: int):
    out, i = [], 0
    while mask:
        if mask & 1:
            out.append(i)
        mask >>= 1
        i += 1
    return out


def act(mask: int, ops):
    """Apply ops = [(creator?, orbital), ...] (product order, the last acts first) to the
    determinant `mask`: returns (sign, new mask), or None when the result vanishes."""
    sign = 1
    for cre, i in reversed(ops):
        occ = (mask >> i) & 1
        if cre == occ:  # creating on an occupied or annihilating an empty orbital
            return None
        if bin(mask & ((1 << i) - 1)).count("1") & 1:
            sign = -sign
        mask ^= 1 << i
    return sign, mask


def element(h, v, gamma: float, a: int, b: int) -> float:
    """<a| H + gamma |b> for two determinants with the same particle number."""
    holes = _bits(b & ~a)   # occupied in b, empty in a
    parts = _bits(a & ~b)   # empty in b, occupied in a
    if len(holes) != len(parts) or len(holes) > 2:
        return 0.0
    common = _bits(a & b)
    total = gamma if a == b else 0.0
    # one-body terms a_i^* a_j
    if len(holes) == 0:
        pairs = [(i, i) for i in common]
    elif len(holes) == 1:
        pairs = [(parts[0], holes[0])]
    else:
        pairs = []
    for i, j in pairs:
        r = act(b, [(1, i), (0, j)])
        if r is not None and r[1] == a:
            total += h[i, j] * r[0]
    # two-body terms a_i^* a_j^* a_k a_l: the annihilated pair {k, l} holds the holes and
    # the created pair {i, j} the particles; the remaining slots take the same orbital of
    # both determinants
    if len(holes) == 2:
        sets = [(parts, holes)]
    elif len(holes) == 1:
        sets = [([parts[0], m], [holes[0], m]) for m in common]
    else:
        sets = [([m1, m2], [m1, m2]) for m1, m2 in itertools.combinations(common, 2)]
    for cr, an in sets:
        for i, j in itertools.permutations(cr):
            for k, l in itertools.permutations(an):
                r = act(b, [(1, i), (1, j), (0, k), (0, l)])
                if r is not None and r[1] == a:
                    total += v[i, j, k, l] * r[0]
    return total


def single_excitations(b: int, L: int):
    return [b ^ (1 << p) ^ (1 << r) for p in _bits(b) for r in range(L) if not (b >> r) & 1]


def double_excitations(b: int, L: int):
    occ = _bits(b)
    emp = [r for r in range(L) if not (b >> r) & 1]
    return [b ^ (1 << p) ^ (1 << q) ^ (1 << r) ^ (1 << s)
            for p, q in itertools.combinations(occ, 2) for r, s in itertools.combinations(emp, 2)]
