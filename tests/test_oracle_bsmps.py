"""Pins of the block-sparse MPS oracle (oracle/bsmps.py) against the dense oracle and
against identities of its own: the MPO against the Hamiltonian applied by its
definition and the rank bound of Thm. opranks; the truncations against the dense
TT-SVD; the H application with a finite intermediate rank against the exact product
(projection identity and error bound); Algorithm 2 against the dense run."""
import math

import numpy as np
import pytest

from oracle import bsmps as B
from oracle import fock, pinvit, precond, tt
from synth import make_problem, random_block_mps, rho_table


def _bmps(L, N, cap, seed, isometric=False):
    rho = rho_table(L, N, cap)
    return B.from_export(L, N, rho, random_block_mps(L, N, rho, seed, isometric))


@pytest.mark.parametrize("kind,L,seed", [("dense", 5, 0), ("dense", 6, 3), ("decayed", 7, 1)])
def test_mpo_equals_hamiltonian(kind, L, seed):
    # the MPO contracted to a 2^L x 2^L matrix equals H + shift * (number operator), with
    # H applied term by term on bit strings (eq. hamil, Jordan-Wigner operators)
    p = make_problem(kind, L, L // 2, seed)
    shift = 0.37
    mpo = B.build_mpo(p.h, p.v, shift)
    eye = np.eye(1 << L)
    ref = fock.apply_h(p.h, p.v, eye) + shift * fock.number_op(eye)
    assert np.abs(mpo.to_dense() - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("L", [6, 8, 10, 12])
def test_mpo_bond_dimension_reaches_the_bound(L):
    # Thm. opranks: ranks at most L^2/2 + 3L/2 + 2, attained in the middle of the chain
    p = make_problem("decayed", L, L // 2, 0)
    mpo = B.build_mpo(p.h, p.v, 0.0)
    w = [mpo.w(m) for m in range(L + 1)]
    bound = L * L // 2 + 3 * L // 2 + 2
    assert max(w) == bound and w[L // 2] == bound
    assert w[0] == w[L] == 1
    # per charge in the middle: q = 0: 2 + n^2, q = +-1: L, q = +-2: n(n-1)/2, n = L/2
    n = L // 2
    q = mpo.q[L // 2]
    assert [int(np.sum(q == c)) for c in (-2, -1, 0, 1, 2)] == [n * (n - 1) // 2, L, 2 + n * n, L, n * (n - 1) // 2]


def test_dot_lincomb_scale_match_dense():
    L, N = 8, 4
    x, y = _bmps(L, N, 6, 1), _bmps(L, N, 5, 2)
    xd, yd = B.to_dense(x), B.to_dense(y)
    assert B.dot(x, y) == pytest.approx(float(xd @ yd), abs=1e-14 * np.linalg.norm(xd) * np.linalg.norm(yd))
    z = B.lincomb(0.3, x, -1.2, y)
    assert np.abs(B.to_dense(z) - (0.3 * xd - 1.2 * yd)).max() <= 1e-14
    assert (z.rho[1:L] == (x.rho + y.rho)[1:L]).all()
    assert np.abs(B.to_dense(B.scale(x, -2.5)) + 2.5 * xd).max() <= 1e-14
    rho, data = B.to_export(x)
    assert np.abs(B.to_dense(B.from_export(L, N, rho, data)) - xd).max() == 0.0


def test_determinant():
    L, N, occ = 7, 3, [0, 3, 5]
    d = B.determinant(L, N, occ)
    assert np.array_equal(B.to_dense(d), fock.determinant(L, occ))
    assert d.max_rank() == 1


def test_right_orthogonalize():
    L, N = 8, 4
    x = _bmps(L, N, 8, 4)
    y = B.right_orthogonalize(x)
    assert np.abs(B.to_dense(y) - B.to_dense(x)).max() <= 1e-13
    for k in range(2, L + 1):
        for n in B.sectors(L, N, k - 1):
            C = np.hstack([y.blk[k][(n, s)] for s in (0, 1) if (n, s) in y.blk[k]])
            assert np.abs(C @ C.T - np.eye(C.shape[0])).max() <= 1e-13


@pytest.mark.parametrize("eps,cap", [(0.0, 1000), (0.05, 1000), (0.0, 4), (0.3, 5), (0.01, 7)])
def test_truncations_match_dense(eps, cap):
    L, N = 8, 4
    z = B.lincomb(1.0, _bmps(L, N, 6, 11), 0.7, _bmps(L, N, 6, 12))
    zd = B.to_dense(z)
    y, cb, _, sv = B.truncate(z, eps, cap)
    yd, rho, cbd, _, _ = tt.truncate(zd, L, N, eps, cap)
    assert np.abs(B.to_dense(y) - yd).max() <= 1e-12
    assert cb == cbd
    assert all(y.rho[k][n] == rho[k][n] for k in range(1, L) for n in rho[k])
    # left-orthogonal output with the norm in the last core
    for k in range(1, L):
        for n in B.sectors(L, N, k):
            M, _ = B._left_fused(y, k, n)
            if M.size:
                assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-12
    yp, cbp, _ = B.truncate_parallel(z, eps, cap)
    ydp, rhop, cbdp, _ = tt.truncate_parallel(zd, L, N, eps, cap)
    assert np.abs(B.to_dense(yp) - ydp).max() <= 1e-12
    assert cbp == cbdp
    assert all(yp.rho[k][n] == rhop[k][n] for k in range(1, L) for n in rhop[k])


def _right_parts(mpo, xr, k):
    """Dense right parts at cut k: the operator's right part from every state b (a matrix
    over the occupations of orbitals k+1..L, orbital k+1 the least significant bit) and
    the right part of xr from every bond index of every sector."""
    L, N = xr.L, xr.N
    # right part of x at cut m: for sector n a matrix (rho(m, n), 2^(L-m))
    R = {L: {N: np.ones((1, 1))}}
    for m in range(L - 1, k - 1, -1):
        R[m] = {}
        for n in B.sectors(L, N, m):
            acc = np.zeros((xr.rho[m][n], 1 << (L - m)))
            for s in (0, 1):
                if (n, s) in xr.blk[m + 1]:
                    # orbital m+1 is the least significant bit of the right index
                    part = xr.blk[m + 1][(n, s)] @ R[m + 1][n + s]
                    acc[:, s::2] += part
            R[m][n] = acc
    # operator right part from cut m: for state b a tensor (2^(L-m) out, 2^(L-m) in)
    O = {L: [np.ones((1, 1))]}
    for m in range(L - 1, k - 1, -1):
        W = mpo.dense_site(m)
        nxt = []
        for b in range(W.shape[0]):
            acc = np.zeros((1 << (L - m), 1 << (L - m)))
            for bp in range(W.shape[1]):
                f = W[b, bp]
                if f.any():
                    acc += np.kron(O[m + 1][bp], f)
            nxt.append(acc)
        O[m] = nxt
    return O[k], R[k]


def test_zipup_exact_equals_product():
    L, N = 8, 4
    p = make_problem("dense", L, N, 0)
    mpo = B.build_mpo(p.h, p.v, p.gamma / N)
    x = _bmps(L, N, 6, 1)
    y, d2, bound = B.zipup(x, mpo, 0)
    ref = fock.apply_h(p.h, p.v, B.to_dense(x), p.gamma)
    assert np.abs(B.to_dense(y) - ref).max() <= 1e-12 * np.abs(ref).max()
    assert d2 == 0.0 and not bound
    # an intermediate rank at least the exact ranks gives the same product
    y2, d2b, b2 = B.zipup(x, mpo, y.max_rank())
    assert np.abs(B.to_dense(y2) - ref).max() <= 1e-12 * np.abs(ref).max()
    assert d2b == 0.0 and not b2


@pytest.mark.parametrize("m_zip", [3, 8, 16])
def test_zipup_finite_rank_is_projection_with_error_bound(m_zip):
    """With a binding m_zip the result is Q Q^T H x for the orthonormal left basis Q of
    its first L-1 cores (Q^T of the error vanishes), and the error obeys
    ||H x - y||^2 = sum_k ||(I - U_k U_k^T) P_k R_k||^2 <= sum_k d_k ||R_k||^2 with d_k the
    weight dropped at site k and R_k the right parts of the panel's columns."""
    L, N = 8, 4
    p = make_problem("dense", L, N, 0)
    mpo = B.build_mpo(p.h, p.v, p.gamma / N)
    x = _bmps(L, N, 6, 1)
    hx = fock.apply_h(p.h, p.v, B.to_dense(x), p.gamma)
    y, d2, bound = B.zipup(x, mpo, m_zip)
    assert bound and d2 > 0
    assert max(y.rho[k].sum() for k in range(1, L)) <= m_zip
    yd = B.to_dense(y)
    err = hx - yd
    # the cores 1..L-1 are left-orthonormal
    for k in range(1, L):
        for n2 in B.sectors(L, N, k):
            M, _ = B._left_fused(y, k, n2)
            if M.size:
                assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-12
    # projection identity: the error is orthogonal to every vector with y's left part
    # and any last core: test with the last core replaced by unit vectors
    for (n, s), blk in y.blk[L].items():
        for r in range(blk.shape[0]):
            z = y.copy()
            for key in z.blk[L]:
                z.blk[L][key] = np.zeros_like(z.blk[L][key])
            z.blk[L][(n, s)][r, 0] = 1.0
            assert abs(float(B.to_dense(z) @ err)) <= 1e-12 * np.linalg.norm(hx)
    assert np.linalg.norm(hx) ** 2 - np.linalg.norm(yd) ** 2 == pytest.approx(np.linalg.norm(err) ** 2,
                                                                            abs=1e-12 * np.linalg.norm(hx) ** 2)
    # error bound: per-site dropped weight times the squared norm of the right parts
    per = []
    B.zipup(x, mpo, m_zip, per_cut=per)
    assert sum(per) == pytest.approx(d2, rel=1e-14)
    xr = B.right_orthogonalize(x)
    bound_sq = 0.0
    for k in range(1, L):
        Rk = _right_part_matrix(mpo, xr, k)
        bound_sq += per[k - 1] * np.linalg.norm(Rk, 2) ** 2
    assert np.linalg.norm(err) ** 2 <= bound_sq * (1 + 1e-10)


def _right_part_matrix(mpo, xr, k):
    """The right parts O_b R_c of all pairs (b, c) at cut k as rows of one matrix: a
    superset of the panel's columns (those with matching charges), so its spectral norm
    bounds theirs."""
    L, N = xr.L, xr.N
    Ok, Rk = _right_parts(mpo, xr, k)
    rows = []
    for b in range(len(Ok)):
        for n in B.sectors(L, N, k):
            for c in range(Rk[n].shape[0]):
                rows.append(Ok[b] @ Rk[n][c])
    return np.array(rows)


def test_expect_matches_dense():
    L, N = 8, 4
    p = make_problem("decayed", L, N, 2)
    mpo = B.build_mpo(p.h, p.v, p.gamma / N)
    a, b = _bmps(L, N, 6, 5), _bmps(L, N, 4, 6)
    ad, bd = B.to_dense(a), B.to_dense(b)
    ref = float(ad @ fock.apply_h(p.h, p.v, bd, p.gamma))
    assert B.expect(a, b, mpo) == pytest.approx(ref, abs=1e-13 * np.linalg.norm(ad) * np.linalg.norm(bd) * 50)
    assert B.expect(a, b, mpo) == pytest.approx(B.expect(b, a, mpo), rel=1e-12)


@pytest.mark.parametrize("eta", [1e-3, 0.1])
def test_apply_s_matches_dense(eta):
    L, N = 8, 4
    p = make_problem("dense", L, N, 0)
    pre = precond.Preconditioner(p.h, p.v, N, p.gamma)
    x = _bmps(L, N, 6, 1)
    sy, cb = B.apply_s(pre, x, eta, 1000)
    sd, cbd, _, _ = precond.apply_sorted(pre, B.to_dense(x), eta, 1000, N)
    assert np.abs(B.to_dense(sy) - sd).max() <= 1e-13
    assert cb == cbd


@pytest.mark.parametrize("kind,L,N,seed,cap,iters,mode", [
    ("dense", 8, 4, 0, 16, 20, "sequential"),
    ("decayed", 10, 5, 1, 8, 12, "sequential"),
    ("dense", 8, 4, 0, 16, 12, "parallel"),
])
def test_run_matches_dense_oracle(kind, L, N, seed, cap, iters, mode):
    """Algorithm 2 on block-sparse MPS with the exact product equals the dense run."""
    p = make_problem(kind, L, N, seed)
    w = fock.lowest_eigs(p.h, p.v, N, p.gamma, k=2)
    delta = w[1] / (w[1] - w[0])
    prm = pinvit.Params(cap=cap, max_iter=iters, tau=1e-12, c=0.5, delta=delta, truncation=mode)
    psi_o, h_o, _ = pinvit.run(p.h, p.v, N, p.gamma, prm)
    psi_b, h_b, _ = B.run(p.h, p.v, N, p.gamma, prm, m_zip=0)
    assert len(h_o) == len(h_b)
    for a, b in zip(h_o, h_b):
        assert abs(a["E"] - b["E"]) <= 1e-10 * abs(a["E"])
        assert a["retries"] == b["retries"]
        assert a["rho"] == pytest.approx(b["rho"], rel=1e-8)
        assert not b["zip_bound"]
    x = B.to_dense(psi_b)
    assert abs(abs(x @ psi_o) / (np.linalg.norm(x) * np.linalg.norm(psi_o)) - 1) <= 1e-10


def test_run_with_binding_m_zip_is_variational_and_never_certified():
    """A binding intermediate rank leaves the iteration variational (every lambda is a
    Rayleigh quotient, above the exact eigenvalue) but uncertified: every row reports
    the flag and the dropped weight, and the run does not stop on its bound, while the
    exact product reaches the same tau."""
    L, N = 6, 3
    p = make_problem("dense", L, N, 0)
    w = fock.lowest_eigs(p.h, p.v, N, p.gamma, k=2)
    prm = pinvit.Params(cap=64, max_iter=40, tau=1e-3, c=0.5, delta=w[1] / (w[1] - w[0]))
    _, hist0, _ = B.run(p.h, p.v, N, p.gamma, prm, m_zip=0)
    assert hist0[-1].get("stop") and len(hist0) < 40 and not any(r["zip_bound"] for r in hist0)
    _, hist, _ = B.run(p.h, p.v, N, p.gamma, prm, m_zip=4)
    assert len(hist) == 40
    for r in hist:
        assert r["lam"] >= w[0] - 1e-10
        assert r["zip_bound"] and r["zip_disc"] > 0 and r["cap_bound"] and not r.get("stop")


def test_stored_L24_runs_under_two_svd_drivers():
    """The stored L = 24 runs (N = 12, cap 128, m_zip 512, 50 iterations) of the oracle with
    LAPACK's divide-and-conquer and QR-iteration SVD drivers: a rounding-level change of
    the same method.  Ranks, retries and flags agree in every iteration; the energies
    agree to rounding for the first 15 iterations and then drift apart at most to the
    1e-5 level, as the binding rank cap amplifies rounding differences (the same profile
    the GPU run shows against the oracle)."""
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    paths = [os.path.join(here, f) for f in ("omps_L24_N12_cap128_mzip512.json",
                                             "omps_L24_N12_cap128_mzip512_qrsvd.json")]
    if not all(os.path.exists(q) for q in paths):
        pytest.skip("stored runs not written")
    a, b = (json.load(open(q))["history"] for q in paths)
    assert len(a) == len(b) == 50
    rel = []
    for ra, rb in zip(a, b):
        for key in ("retries", "cap_bound", "zip_bound", "max_rank"):
            assert ra[key] == rb[key], (ra["it"], key)
        rel.append(abs(ra["E"] - rb["E"]) / abs(rb["E"]))
    assert max(rel[:16]) <= 1e-13
    assert max(rel) <= 1e-4
