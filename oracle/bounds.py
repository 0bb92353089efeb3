"""A-posteriori quantities of Section 5.4 and the Ritz step of Rem. omegamin (oracle)."""
from __future__ import annotations

import math

import numpy as np


def b_delta(rho: float, delta: float) -> float:
    """b_delta(rho) of eq. bbetarho; requires rho^2 <= 1/(4 delta (delta-1))."""
    disc = 1.0 - 4.0 * (delta - 1.0) * delta * rho * rho
    if disc < 0.0:
        return math.nan
    return 2.0 * delta / (1.0 + 2.0 * delta * rho * rho + math.sqrt(disc))


def eigvec_error_bound(rho: float, delta: float) -> float:
    """2 sin(arcsin(sqrt(delta b_delta(rho)) rho)/2) of eq. everrbound (nan outside
    the domain of Lemma lambdaqbound)."""
    if rho * rho > 1.0 / (4.0 * delta * (delta - 1.0)):
        return math.nan
    arg = math.sqrt(delta * b_delta(rho, delta)) * rho
    if arg > 1.0:
        return math.nan
    return 2.0 * math.sin(0.5 * math.asin(arg))


def rel_eig_bound(rho: float, delta: float) -> float:
    """Relative eigenvalue bound of eq. releigerr."""
    b = b_delta(rho, delta)
    return b * rho * rho / (1.0 - b * rho * rho)


def gap_delta(l1: float, l2: float) -> float:
    return l2 / (l2 - l1)


def ritz2(hm: np.ndarray, mm: np.ndarray):
    """Lower eigenpair of the 2x2 pencil hm v = lam mm v (Rem. omegamin).

    Closed form: det(hm - lam mm) = 0 is the quadratic a lam^2 + b lam + c = 0 with
    a = det(mm), b = -(hm00 mm11 + hm11 mm00 - 2 hm01 mm01), c = det(hm); the lower
    root is taken and v is normalised to v^T mm v = 1 with v_0 > 0."""
    a = mm[0, 0] * mm[1, 1] - mm[0, 1] ** 2
    b = -(hm[0, 0] * mm[1, 1] + hm[1, 1] * mm[0, 0] - 2.0 * hm[0, 1] * mm[0, 1])
    c = hm[0, 0] * hm[1, 1] - hm[0, 1] ** 2
    disc = max(b * b - 4.0 * a * c, 0.0)
    # numerically stable smaller root
    if b < 0:
        q = -0.5 * (b - math.sqrt(disc))
        r1, r2 = q / a, c / q
    else:
        q = -0.5 * (b + math.sqrt(disc))
        r1, r2 = c / q, q / a
    lam = min(r1, r2)
    k = hm - lam * mm
    # null vector of the 2x2 singular matrix k: take the better-conditioned row
    if abs(k[0, 0]) + abs(k[0, 1]) >= abs(k[1, 0]) + abs(k[1, 1]):
        v = np.array([-k[0, 1], k[0, 0]])
    else:
        v = np.array([k[1, 1], -k[1, 0]])
    nrm = math.sqrt(float(v @ mm @ v))
    v = v / nrm
    if v[0] < 0 or (v[0] == 0 and v[1] < 0):
        v = -v
    return lam, v


def delta_a(rho: float, q: float) -> float:
    """Root Delta of sqrt(1-Delta^2) - rho Delta = q (Alg. 2, iterate truncation)."""
    return (-q * rho + math.sqrt(q * q * rho * rho + (1.0 + rho * rho) * (1.0 - q * q))) / (1.0 + rho * rho)
