"""Writes the stored Algorithm 2 histories of the block-sparse MPS oracle that the GPU
parity tests compare with (runs too long to repeat inside a test).

Usage:  python tests/golden/make_omps_runs.py [--qr-svd] [name ...]   (default: every run below)

--qr-svd takes every SVD of the oracle with LAPACK's QR-iteration driver instead of its
divide-and-conquer one, a rounding-level change of the same method, and writes
omps_<name>_qrsvd.json: how far two correct runs of the method drift apart under the
binding rank cap.

Each run writes tests/golden/omps_<name>.json: the parameters and, per iteration, the
energy, Rayleigh quotient, residual bound, norms, tolerance, retries, flags and the block
table of the new iterate.  Only the oracle (oracle.bsmps) and the input generators
(synth) are called.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bsmps, pinvit  # noqa: E402
from synth import make_problem  # noqa: E402

# the plain float64 workload at L = 24: decayed integrals seed 0, N = 12, rank cap 128,
# the exact H application (m_zip <= 0: intermediate ranks up to the full sector
# dimensions, at most 4096 per bond), sequential truncation, 50 iterations
# the same with the intermediate rank of the H application capped at 512 (the zip cap of the
# L = 48 benchmark), which keeps every Gram matrix of the GPU path within order 1024
RUNS = {
    "L24_N12_cap128_exact": dict(kind="decayed", L=24, N=12, seed=0, cap=128, m_zip=0, iters=50,
                                 truncation="sequential", c=0.5, delta=10.0, tau=0.0),
    "L24_N12_cap128_mzip512": dict(kind="decayed", L=24, N=12, seed=0, cap=128, m_zip=512, iters=50,
                                   truncation="sequential", c=0.5, delta=10.0, tau=0.0),
}


def make(name: str, qr_svd: bool = False) -> str:
    cfg = RUNS[name]
    if qr_svd:
        import scipy.linalg
        bsmps._svd = lambda M: scipy.linalg.svd(M, full_matrices=False, lapack_driver="gesvd")
        name = name + "_qrsvd"
    p = make_problem(cfg["kind"], cfg["L"], cfg["N"], cfg["seed"])
    prm = pinvit.Params(cap=cfg["cap"], max_iter=cfg["iters"], tau=cfg["tau"], c=cfg["c"],
                        delta=cfg["delta"], truncation=cfg["truncation"])
    out = os.path.join(HERE, f"omps_{name}.json")
    rows = []
    t0 = time.time()

    def record(rec, psi):
        rows.append(rec)
        print(f"# {name}: iteration {rec['it']} E={rec['E']:.12f} retries={rec['retries']} "
              f"max_rank={rec['max_rank']} ({time.time() - t0:.0f}s)", flush=True)

    _, hist, _ = bsmps.run(p.h, p.v, cfg["N"], p.gamma, prm, m_zip=cfg["m_zip"], callback=record)
    keep = ("it", "lam", "E", "rho", "r_norm", "s_norm", "eta", "retries", "cap_bound", "zip_bound",
            "zip_disc", "max_rank", "lam_star", "eta_psi")
    data = {"name": name, "config": cfg, "gamma": p.gamma,
            "history": [{**{k: (bool(r[k]) if isinstance(r[k], bool) else r[k]) for k in keep if k in r},
                         "rho_tab": [[int(v) for v in row] for row in r["rho_tab"]] if "rho_tab" in r else None}
                        for r in hist]}
    with open(out, "w") as f:
        json.dump(data, f, indent=0)
    return out


if __name__ == "__main__":
    args = sys.argv[1:]
    qr = "--qr-svd" in args
    names = [a for a in args if a != "--qr-svd"]
    for name in (names or list(RUNS)):
        print(make(name, qr), flush=True)
