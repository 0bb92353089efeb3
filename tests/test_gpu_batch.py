"""Batched independent problems (pv_run_batch): several Hamiltonians of different size,
rank cap and truncation mode run concurrently, each on its own context; every result must
equal that of the same context run alone (the kernels are deterministic), and a bad member
fails the call without hiding the error."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

native = pytest.importorskip("paper_2604_16118_amd.native")
from synth import make_problem  # noqa: E402

PROBLEMS = [  # (kind, L, N, seed, params)
    ("dense", 8, 4, 0, dict(rank_cap=16, max_iter=4, tau=0.0, truncation=0)),
    ("decayed", 10, 5, 1, dict(rank_cap=24, max_iter=4, tau=0.0, truncation=1, m_zip=24)),
    ("decayed", 12, 6, 2, dict(rank_cap=32, max_iter=3, tau=0.0, truncation=1, m_zip=32)),
    ("dense", 9, 3, 3, dict(rank_cap=8, max_iter=5, tau=0.0, truncation=0)),
    ("decayed", 16, 8, 4, dict(rank_cap=48, max_iter=3, tau=0.0, truncation=1, m_zip=48)),
]


@pytest.fixture(scope="module")
def contexts():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctxs = []
    for kind, L, N, seed, _ in PROBLEMS:
        p = make_problem(kind, L, N, seed)
        c = native.Context(0)
        c.set_hamiltonian(p.h, p.v, N, p.gamma)
        ctxs.append(c)
    yield ctxs
    for c in ctxs:
        c.close()


def test_batch_equals_individual_runs(contexts):
    params = [pr for *_, pr in PROBLEMS]
    alone = [c.run(**pr)[0] for c, pr in zip(contexts, params)]
    for rep in range(2):
        batch = native.run_batch(contexts, params)
        for a, b in zip(alone, batch):
            assert b["iterations"] == a["iterations"]
            assert b["energy"] == a["energy"]
            assert b["rho"] == a["rho"]


def test_batch_rejects_repeated_context(contexts):
    with pytest.raises(native.PvError):
        native.run_batch([contexts[0], contexts[0]], [PROBLEMS[0][4]] * 2)


def test_batch_reports_failed_member(contexts):
    bare = native.Context(0)  # no Hamiltonian: that member fails, the others still run
    try:
        with pytest.raises(native.PvError, match="problem 1"):
            native.run_batch([contexts[0], bare], [PROBLEMS[0][4]] * 2)
    finally:
        bare.close()
