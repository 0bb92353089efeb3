"""ctypes binding of libpinvit.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/pinvit.h with the same
name; arrays are passed as NumPy float64/int32 host buffers.  The library must have
been built (``python -m paper_2604_16118_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpinvit.so")

STATUS = {0: "PV_OK", -1: "PV_EINVAL", -2: "PV_ENOMEM", -3: "PV_EDEVICE", -4: "PV_ENOTSPD",
          -5: "PV_ENOCONV", -6: "PV_ESTATE"}

# names exported by include/pinvit.h
EXPORTS = [
    "pv_last_error", "pv_create", "pv_destroy", "pv_set_hamiltonian", "pv_precond_info",
    "pv_mps_create", "pv_mps_determinant", "pv_mps_layout", "pv_mps_download", "pv_mps_free",
    "pv_set_truncation", "pv_set_tridiag_steps", "pv_dot", "pv_expect_h", "pv_lincomb", "pv_round", "pv_apply_h", "pv_apply_s", "pv_run", "pv_run_outer", "pv_run_subspace", "pv_run_subspace_joint", "pv_run_zform", "pv_run_batch",
    "pv_set_correction", "pv_learned_correction", "pv_learned_train", "pv_learned_train_solves",
    "pv_set_learned_network", "pv_solve_h", "pv_mps_amplitudes",
    "pv_timers", "pv_timer_name", "pv_timers_reset", "pv_set_timer_mask", "pv_set_timer_sampling", "pv_sym_eig", "pv_sym_eig_top", "pv_sym_eig_noalloc", "pv_gemm", "pv_cholesky", "pv_mpo_bond_dims", "pv_mpo_dense",
    "pv_mfma_f64_rate", "pv_set_gemm_tiles", "pv_gemm_tune_table", "pv_gemm_tune_clear",
    "pv_set_learned_judge", "pv_learned_judge_counts", "pv_gemm_tune_load",
]


MLP_WIDTH = 256
MLP_PARAMS = MLP_WIDTH * 6 + MLP_WIDTH + MLP_WIDTH * MLP_WIDTH + MLP_WIDTH + MLP_WIDTH + 1


class PvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("rank_cap", C.c_int), ("m_zip", C.c_int), ("max_iter", C.c_int),
                ("tau", C.c_double), ("c0", C.c_double), ("c", C.c_double),
                ("delta", C.c_double), ("eps_num", C.c_double), ("t_eig", C.c_double),
                ("c_lower", C.c_double), ("c_upper", C.c_double), ("max_retries", C.c_int),
                ("precision", C.c_int), ("truncation", C.c_int), ("resume_eta", C.c_double),
                ("resume_s", C.c_double),
                ("resume_s2", C.c_double)]


class Iter(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("energy", C.c_double), ("rho", C.c_double),
                ("bound", C.c_double), ("r_norm", C.c_double), ("s_norm", C.c_double),
                ("eta_res", C.c_double), ("lambda_star", C.c_double), ("eta_psi", C.c_double),
                ("seconds", C.c_double), ("retries", C.c_int), ("cap_bound", C.c_int),
                ("max_rank", C.c_int), ("stopped", C.c_int), ("zip_bound", C.c_int),
                ("zip_discard", C.c_double)]


class OuterIter(C.Structure):
    _fields_ = [("eta", C.c_double), ("tau", C.c_double), ("lambda_", C.c_double),
                ("energy", C.c_double), ("rho", C.c_double), ("rel_bound", C.c_double),
                ("trunc_eps", C.c_double), ("inner_iterations", C.c_int), ("cap_bound", C.c_int),
                ("max_rank", C.c_int), ("stopped", C.c_int)]


SUBSPACE_MAX_D = 8
TRIDIAG_STEPS_DEFAULT = 1 << 30  # PV_TRIDIAG_STEPS_DEFAULT
# float64 GEMM tile modes (PV_GEMM_TILES_*)
GEMM_TILES = {"rule": 0, "tune": 1, "table": 2, "small": 3, "large": 4}


class SubspaceIter(C.Structure):
    _fields_ = [("lambda_", C.c_double * SUBSPACE_MAX_D), ("energy", C.c_double * SUBSPACE_MAX_D),
                ("rho", C.c_double * SUBSPACE_MAX_D), ("s_norm", C.c_double * SUBSPACE_MAX_D),
                ("lambda_star", C.c_double * SUBSPACE_MAX_D), ("bound", C.c_double),
                ("eta_res", C.c_double), ("eta_psi", C.c_double), ("seconds", C.c_double),
                ("retries", C.c_int), ("cap_bound", C.c_int), ("max_rank", C.c_int), ("stopped", C.c_int)]


class Result(C.Structure):
    _fields_ = [("energy", C.c_double), ("lambda_", C.c_double), ("rho", C.c_double),
                ("bound", C.c_double), ("eta_res", C.c_double), ("s_last", C.c_double),
                ("s_prev", C.c_double), ("iterations", C.c_int), ("converged", C.c_int)]


_lib = None


def lib():
    """Load the library (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: run `python -m paper_2604_16118_amd.build`")
        L = C.CDLL(LIB_PATH)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
        L.pv_last_error.restype = C.c_char_p
        L.pv_timer_name.restype = C.c_char_p
        L.pv_destroy.restype = None
        L.pv_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]
        L.pv_destroy.argtypes = [C.c_void_p]
        L.pv_set_hamiltonian.argtypes = [C.c_void_p, C.c_int, C.c_int, dp, dp, C.c_double]
        L.pv_precond_info.argtypes = [C.c_void_p, dp, ip]
        L.pv_mps_create.argtypes = [C.c_void_p, ip, dp, C.c_size_t, ip]
        L.pv_mps_determinant.argtypes = [C.c_void_p, ip, ip]
        L.pv_mps_layout.argtypes = [C.c_void_p, C.c_int, ip, C.POINTER(C.c_size_t)]
        L.pv_mps_download.argtypes = [C.c_void_p, C.c_int, dp, C.c_size_t]
        L.pv_mps_free.argtypes = [C.c_void_p, C.c_int]
        L.pv_set_truncation.argtypes = [C.c_void_p, C.c_int]
        L.pv_set_tridiag_steps.argtypes = [C.c_void_p, C.c_int]
        L.pv_dot.argtypes = [C.c_void_p, C.c_int, C.c_int, dp]
        L.pv_expect_h.argtypes = [C.c_void_p, C.c_int, C.c_int, dp]
        L.pv_lincomb.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_double, C.c_int, ip]
        L.pv_round.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int, ip, ip]
        L.pv_apply_h.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_int, ip, ip,
                                 C.POINTER(C.c_double)]
        L.pv_apply_s.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int, ip, ip]
        L.pv_run.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int, C.POINTER(Result),
                             C.POINTER(Iter), C.c_int, ip]
        L.pv_run_outer.argtypes = [C.c_void_p, C.POINTER(Params), C.c_double, C.c_double, C.c_int,
                                   C.POINTER(Result), C.POINTER(OuterIter), C.c_int, ip]
        L.pv_run_zform.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int, C.POINTER(Result),
                                   C.POINTER(Iter), C.c_int, ip]
        L.pv_run_subspace.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int, ip, C.POINTER(Result),
                                      C.POINTER(SubspaceIter), C.c_int, ip]
        L.pv_run_subspace_joint.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int, C.c_int, C.POINTER(Result),
                                            C.POINTER(SubspaceIter), C.c_int, ip]
        L.pv_run_batch.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(Params), C.POINTER(Result), ip]
        L.pv_timers.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, ip]
        L.pv_timers_reset.argtypes = [C.c_void_p]
        L.pv_set_timer_mask.argtypes = [C.c_void_p, C.c_uint32]
        L.pv_set_timer_sampling.argtypes = [C.c_void_p, C.c_uint32, C.c_int]
        L.pv_sym_eig.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, C.c_int]
        L.pv_sym_eig_top.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, C.c_int]
        L.pv_sym_eig_noalloc.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.pv_gemm.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, dp, C.c_int, C.c_int, dp, C.c_int, C.c_int,
                              dp, C.c_int, C.c_double, C.c_double, C.c_int]
        L.pv_cholesky.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.pv_mfma_f64_rate.argtypes = [C.c_void_p, dp]
        L.pv_set_gemm_tiles.argtypes = [C.c_void_p, C.c_int]
        L.pv_set_learned_judge.argtypes = [C.c_void_p, C.c_int]
        L.pv_learned_judge_counts.argtypes = [C.c_void_p, ip, ip]
        L.pv_gemm_tune_table.argtypes = [dp, C.c_int, ip]
        L.pv_gemm_tune_clear.argtypes = []
        L.pv_gemm_tune_load.argtypes = [dp, C.c_int]
        fp, up = C.POINTER(C.c_float), C.POINTER(C.c_uint64)
        L.pv_learned_train_solves.argtypes = [C.c_void_p, fp, C.c_int, up, C.c_int, dp, dp, C.c_int, C.c_float,
                                              dp, dp]
        L.pv_set_learned_network.argtypes = [C.c_void_p, fp, C.c_int]
        L.pv_solve_h.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int, ip, ip, dp]
        L.pv_mps_amplitudes.argtypes = [C.c_void_p, C.c_int, up, C.c_int, dp]
        L.pv_mpo_bond_dims.argtypes = [C.c_int, dp, dp, ip, ip]
        L.pv_mpo_dense.argtypes = [C.c_int, dp, dp, C.c_double, dp]
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise PvError(st, lib().pv_last_error().decode())


def make_params(rank_cap, max_iter, tau=1e-10, c=0.5, delta=10.0, m_zip=0, c0=0.1, eps_num=0.0,
                t_eig=0.5, c_lower=0.0, c_upper=0.0, max_retries=30, precision=0, truncation=0,
                resume=None):
    """pv_params of one run (defaults as in Context.run)."""
    r = resume or {}
    return Params(rank_cap, m_zip, max_iter, tau, c0, c, delta, eps_num, t_eig, c_lower,
                  c_upper, max_retries, precision, truncation, r.get("eta_res", 0.0),
                  r.get("s_last", 0.0), r.get("s_prev", 0.0))


def run_batch(contexts, params):
    """pv_run_batch: every context (Hamiltonian set) runs from its determinant with its own
    keyword arguments (those of Context.run), concurrently.  Returns one result dict per
    problem."""
    n = len(contexts)
    if len(params) != n:
        raise ValueError("one parameter set per context")
    ptrs = (C.c_void_p * max(n, 1))(*[ctx._p for ctx in contexts])
    prm = (Params * max(n, 1))(*[make_params(**p) for p in params])
    res = (Result * max(n, 1))()
    st = (C.c_int * max(n, 1))()
    _check(lib().pv_run_batch(ptrs, n, prm, res, st))
    return [dict(energy=r.energy, lam=r.lambda_, rho=r.rho, bound=r.bound, iterations=r.iterations,
                 converged=bool(r.converged)) for r in res[:n]]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def gemm_tune_table():
    """The GEMM tile autotuner's table (pv_gemm_tune_table): one dict per key."""
    n = C.c_int()
    _check(lib().pv_gemm_tune_table(None, 0, C.byref(n)))
    rows = np.zeros(max(n.value, 1) * 9)
    _check(lib().pv_gemm_tune_table(_dp(rows), n.value, C.byref(n)))
    names = ("device", "prec", "tiles_log2", "k_log2", "choice", "n64", "n32", "tflops64", "tflops32")
    out = []
    for r in rows[: 9 * n.value].reshape(-1, 9):
        d = dict(zip(names, r.tolist()))
        for k in names[:7]:
            d[k] = int(d[k])
        out.append(d)
    return out


def gemm_tune_load(rows):
    """Load tuner rows (dicts as gemm_tune_table returns them) into the table
    (pv_gemm_tune_load)."""
    names = ("device", "prec", "tiles_log2", "k_log2", "choice", "n64", "n32", "tflops64", "tflops32")
    a = np.array([[float(r[k]) for k in names] for r in rows], dtype=np.float64).reshape(-1, 9)
    a = np.ascontiguousarray(a)
    _check(lib().pv_gemm_tune_load(_dp(a) if len(rows) else None, len(rows)))


def gemm_tune_clear():
    """Empty the GEMM tile autotuner's table (pv_gemm_tune_clear)."""
    _check(lib().pv_gemm_tune_clear())


def mpo_bond_dims(h, v):
    L = h.shape[0]
    h, v = _f64(h), _f64(v)
    dims = np.zeros(L + 1, np.int32)
    qd = np.zeros((L + 1) * 5, np.int32)
    _check(lib().pv_mpo_bond_dims(L, _dp(h), _dp(v), _ip(dims), _ip(qd)))
    return dims, qd.reshape(L + 1, 5)


def mpo_dense(h, v, diag_shift=0.0):
    L = h.shape[0]
    h, v = _f64(h), _f64(v)
    out = np.zeros((1 << L, 1 << L))
    _check(lib().pv_mpo_dense(L, _dp(h), _dp(v), float(diag_shift), _dp(out)))
    return out


class Context:
    """One library context (device memory, stream, Hamiltonian, MPS handles)."""

    def __init__(self, device: int = 0, stream: int = 0):
        """stream: address of a hipStream_t of the caller (e.g. torch.cuda.Stream's
        cuda_stream) that the context launches on, or 0 for its own."""
        self._p = C.c_void_p()
        _check(lib().pv_create(C.byref(self._p), device, C.c_void_p(stream or None)))
        self.L = self.N = None

    def close(self):
        if self._p:
            lib().pv_destroy(self._p)
            self._p = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_hamiltonian(self, h, v, N, gamma):
        h, v = _f64(h), _f64(v)
        L = h.shape[0]
        _check(lib().pv_set_hamiltonian(self._p, L, N, _dp(h), _dp(v), float(gamma)))
        self.L, self.N, self.gamma = L, N, float(gamma)

    def precond_info(self):
        out = np.zeros(7)
        mr = np.zeros(2, np.int32)
        _check(lib().pv_precond_info(self._p, _dp(out), _ip(mr)))
        keys = ["t_min", "t_max", "T", "h", "alpha0", "s_min", "s_max"]
        d = dict(zip(keys, out.tolist()))
        d["m_minus"], d["m_plus"] = int(mr[0]), int(mr[1])
        return d

    def mps_create(self, rho, data):
        rho = np.ascontiguousarray(rho, dtype=np.int32)
        data = _f64(data)
        h = C.c_int()
        _check(lib().pv_mps_create(self._p, _ip(rho), _dp(data), data.size, C.byref(h)))
        return h.value

    def mps_determinant(self, occupied):
        occ = np.ascontiguousarray(occupied, dtype=np.int32)
        h = C.c_int()
        _check(lib().pv_mps_determinant(self._p, _ip(occ), C.byref(h)))
        return h.value

    def mps_layout(self, handle):
        rho = np.zeros((self.L + 1, self.N + 1), np.int32)
        n = C.c_size_t()
        _check(lib().pv_mps_layout(self._p, handle, _ip(rho), C.byref(n)))
        return rho, n.value

    def mps_download(self, handle):
        rho, n = self.mps_layout(handle)
        data = np.zeros(n)
        _check(lib().pv_mps_download(self._p, handle, _dp(data), n))
        return rho, data

    def mps_free(self, handle):
        _check(lib().pv_mps_free(self._p, handle))

    def set_truncation(self, mode):
        _check(lib().pv_set_truncation(self._p, int(mode)))

    def set_learned_judge(self, on):
        """Per-step judge of a corrected S against the plain S (pv_set_learned_judge)."""
        _check(lib().pv_set_learned_judge(self._p, int(bool(on))))

    def learned_judge_counts(self):
        """(steps won by the plain S, steps won by the corrected S) in the last run."""
        a, b = C.c_int(), C.c_int()
        _check(lib().pv_learned_judge_counts(self._p, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_gemm_tiles(self, mode):
        """Tile shape of the float64 GEMM: "rule", "tune", "table", "small" or "large"
        (pv_set_gemm_tiles)."""
        _check(lib().pv_set_gemm_tiles(self._p, GEMM_TILES[mode] if isinstance(mode, str) else int(mode)))

    def set_tridiag_steps(self, max_problems):
        """Eigensolver batches of at most max_problems matrices use the step-per-launch
        reduction, larger ones the panel kernel (pv_set_tridiag_steps)."""
        _check(lib().pv_set_tridiag_steps(self._p, int(max_problems)))

    def dot(self, a, b):
        out = C.c_double()
        _check(lib().pv_dot(self._p, a, b, C.byref(out)))
        return out.value

    def energy(self, h):
        """<h|H_gamma|h>/<h|h> - gamma (float64 sweeps on the device)."""
        return self.expect_h(h, h) / self.dot(h, h) - self.gamma

    def expect_h(self, bra, ket):
        out = C.c_double()
        _check(lib().pv_expect_h(self._p, bra, ket, C.byref(out)))
        return out.value

    def lincomb(self, a, x, b, y):
        out = C.c_int()
        _check(lib().pv_lincomb(self._p, float(a), x, float(b), y, C.byref(out)))
        return out.value

    def round(self, x, eps, cap):
        out, cb = C.c_int(), C.c_int()
        _check(lib().pv_round(self._p, x, float(eps), int(cap), C.byref(out), C.byref(cb)))
        return out.value, bool(cb.value)

    def apply_h(self, x, eps, cap, m_zip=0, with_discard=False):
        """(handle, cap_bound) of trunc(H x); with_discard also returns the weight m_zip
        dropped (pv_apply_h's zip_discard)."""
        out, cb, zd = C.c_int(), C.c_int(), C.c_double()
        _check(lib().pv_apply_h(self._p, x, float(eps), int(cap), int(m_zip), C.byref(out), C.byref(cb),
                                C.byref(zd)))
        if with_discard:
            return out.value, bool(cb.value), zd.value
        return out.value, bool(cb.value)

    def apply_s(self, x, eta, cap):
        out, cb = C.c_int(), C.c_int()
        _check(lib().pv_apply_s(self._p, x, float(eta), int(cap), C.byref(out), C.byref(cb)))
        return out.value, bool(cb.value)

    def run(self, rank_cap, max_iter, tau=1e-10, c=0.5, delta=10.0, m_zip=0, c0=0.1,
            eps_num=0.0, t_eig=0.5, c_lower=0.0, c_upper=0.0, max_retries=30, start=-1,
            precision=0, truncation=0, resume=None):
        prm = make_params(rank_cap, max_iter, tau, c, delta, m_zip, c0, eps_num, t_eig, c_lower,
                          c_upper, max_retries, precision, truncation, resume)
        res = Result()
        hist = (Iter * max(max_iter, 1))()
        psi = C.c_int()
        _check(lib().pv_run(self._p, C.byref(prm), int(start), C.byref(res), hist,
                            max(max_iter, 1), C.byref(psi)))
        rows = []
        for i in range(res.iterations):
            r = hist[i]
            rows.append(dict(lam=r.lambda_, E=r.energy, rho=r.rho, bound=r.bound, r_norm=r.r_norm,
                             s_norm=r.s_norm, eta=r.eta_res, lam_star=r.lambda_star,
                             eta_psi=r.eta_psi, seconds=r.seconds, retries=r.retries,
                             cap_bound=bool(r.cap_bound), max_rank=r.max_rank,
                             stop=bool(r.stopped), zip_bound=bool(r.zip_bound),
                             zip_disc=r.zip_discard))
        return dict(energy=res.energy, lam=res.lambda_, rho=res.rho, bound=res.bound,
                    iterations=res.iterations, converged=bool(res.converged),
                    eta_res=res.eta_res, s_last=res.s_last, s_prev=res.s_prev), rows, psi.value

    def run_outer(self, alpha=1.0, tol=1e-8, max_outer=20, **kw):
        """Algorithm 3 (pv_run_outer); keyword arguments as in run (max_iter: per outer step).
        Returns (result dict, outer-step rows, handle of the final iterate)."""
        kw.setdefault("max_iter", 50)
        prm = make_params(**kw)
        res = Result()
        hist = (OuterIter * max_outer)()
        psi = C.c_int()
        _check(lib().pv_run_outer(self._p, C.byref(prm), float(alpha), float(tol), int(max_outer),
                                  C.byref(res), hist, int(max_outer), C.byref(psi)))
        rows = [dict(eta=h.eta, tau=h.tau, lam=h.lambda_, E=h.energy, rho=h.rho, rel_bound=h.rel_bound,
                     trunc_eps=h.trunc_eps, inner=h.inner_iterations, cap_bound=bool(h.cap_bound),
                     max_rank=h.max_rank, stop=bool(h.stopped)) for h in hist[:res.iterations]]
        return dict(energy=res.energy, lam=res.lambda_, rho=res.rho, steps=res.iterations,
                    converged=bool(res.converged)), rows, psi.value

    def set_correction(self, delta=None):
        """Learned correction Delta (L x (N+1)) of the preconditioner diagonal, or None to
        clear it (pv_set_correction)."""
        if delta is None:
            _check(lib().pv_set_correction(self._p, None))
            return
        d = np.ascontiguousarray(delta, dtype=np.float64).reshape(-1)
        if d.size != self.L * (self.N + 1):
            raise ValueError("correction must have L (N+1) entries")
        _check(lib().pv_set_correction(self._p, d.ctypes.data_as(C.POINTER(C.c_double))))

    def learned_correction(self, params, psi=-1):
        """Delta (L x (N+1)) of the network with float32 parameters `params` for the iterate
        psi (-1: the start determinant) (pv_learned_correction)."""
        w = np.ascontiguousarray(params, dtype=np.float32)
        if w.size != MLP_PARAMS:
            raise ValueError(f"params must have {MLP_PARAMS} entries")
        out = np.zeros(self.L * (self.N + 1))
        _check(lib().pv_learned_correction(self._p, w.ctypes.data_as(C.POINTER(C.c_float)), int(psi),
                                           out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(self.L, self.N + 1)

    def learned_train(self, params, masks, steps, lr=1e-3, psi=-1, want_grad=False):
        """Adam steps on the diagonal misfit over the determinants `masks` (uint64)
        (pv_learned_train).  Returns (new float32 parameters, losses (steps + 1), gradient at
        the final parameters or None)."""
        w = np.array(params, dtype=np.float32, copy=True)
        if w.size != MLP_PARAMS:
            raise ValueError(f"params must have {MLP_PARAMS} entries")
        m = np.ascontiguousarray(masks, dtype=np.uint64)
        loss = np.zeros(int(steps) + 1)
        grad = np.zeros(MLP_PARAMS) if want_grad else None
        _check(lib().pv_learned_train(self._p, w.ctypes.data_as(C.POINTER(C.c_float)), int(psi),
                                      m.ctypes.data_as(C.POINTER(C.c_uint64)), int(m.size), int(steps),
                                      C.c_float(lr), loss.ctypes.data_as(C.POINTER(C.c_double)),
                                      grad.ctypes.data_as(C.POINTER(C.c_double)) if want_grad else None))
        return w, loss, grad

    def learned_train_solves(self, params, masks, rvals, tvals, steps, lr=1e-3, psi=-1, want_grad=False):
        """Adam steps on the solve form of the misfit (pv_learned_train_solves): the
        residual values rvals and exact-solve values tvals at the determinants masks.
        Returns (new float32 parameters, losses (steps + 1), gradient or None)."""
        w = np.array(params, dtype=np.float32, copy=True)
        if w.size != MLP_PARAMS:
            raise ValueError(f"params must have {MLP_PARAMS} entries")
        m = np.ascontiguousarray(masks, dtype=np.uint64)
        rv, tv = _f64(rvals), _f64(tvals)
        if rv.size != m.size or tv.size != m.size:
            raise ValueError("one residual and one solve value per sample")
        loss = np.zeros(int(steps) + 1)
        grad = np.zeros(MLP_PARAMS) if want_grad else None
        _check(lib().pv_learned_train_solves(self._p, w.ctypes.data_as(C.POINTER(C.c_float)), int(psi),
                                             m.ctypes.data_as(C.POINTER(C.c_uint64)), int(m.size), _dp(rv), _dp(tv),
                                             int(steps), C.c_float(lr), loss.ctypes.data_as(C.POINTER(C.c_double)),
                                             grad.ctypes.data_as(C.POINTER(C.c_double)) if want_grad else None))
        return w, loss, grad

    def set_learned_network(self, params=None, refresh=1):
        """Attach a network to the runs (pv_set_learned_network); None detaches it."""
        if params is None:
            _check(lib().pv_set_learned_network(self._p, None, 0))
            return
        w = np.ascontiguousarray(params, dtype=np.float32)
        if w.size != MLP_PARAMS:
            raise ValueError(f"params must have {MLP_PARAMS} entries")
        _check(lib().pv_set_learned_network(self._p, w.ctypes.data_as(C.POINTER(C.c_float)), int(refresh)))

    def solve_h(self, b, rel_tol=1e-10, max_iter=200):
        """(handle, iterations, relative residual) of x = (H + gamma)^{-1} b (pv_solve_h)."""
        out, it, rr = C.c_int(), C.c_int(), C.c_double()
        _check(lib().pv_solve_h(self._p, int(b), float(rel_tol), int(max_iter), C.byref(out), C.byref(it),
                                C.byref(rr)))  # argtypes convert the Python numbers
        return out.value, it.value, rr.value

    def amplitudes(self, handle, masks):
        m = np.ascontiguousarray(masks, dtype=np.uint64)
        out = np.zeros(m.size)
        _check(lib().pv_mps_amplitudes(self._p, int(handle), m.ctypes.data_as(C.POINTER(C.c_uint64)), int(m.size),
                                       _dp(out)))
        return out

    def run_zform(self, start=-1, **kw):
        """Algorithm 2 on the variable x (pv_run_zform); keyword arguments as in run.  Returns
        (result dict, rows, handle of the final iterate)."""
        kw.setdefault("max_iter", 20)
        n = max(kw["max_iter"], 1)
        prm = make_params(**kw)
        res = Result()
        hist = (Iter * n)()
        x = C.c_int()
        _check(lib().pv_run_zform(self._p, C.byref(prm), int(start), C.byref(res), hist, n, C.byref(x)))
        rows = [dict(lam=r.lambda_, E=r.energy, rho=r.rho, bound=r.bound, r_norm=r.r_norm, eta=r.eta_res,
                     lam_star=r.lambda_star, eta_in=r.eta_psi, seconds=r.seconds, retries=r.retries,
                     cap_bound=bool(r.cap_bound), max_rank=r.max_rank, stop=bool(r.stopped))
                for r in hist[:res.iterations]]
        return dict(energy=res.energy, lam=res.lambda_, rho=res.rho, bound=res.bound,
                    iterations=res.iterations, converged=bool(res.converged)), rows, x.value

    def run_subspace(self, D, starts=None, **kw):
        """Algorithm 4 (pv_run_subspace) on D columns; keyword arguments as in run.  Returns
        (result dict of column 1, rows, handles of the D final columns)."""
        if not 1 <= D <= SUBSPACE_MAX_D:
            raise ValueError(f"D must be in 1..{SUBSPACE_MAX_D}")
        kw.setdefault("max_iter", 20)
        n = max(kw["max_iter"], 1)
        prm = make_params(**kw)
        res = Result()
        hist = (SubspaceIter * n)()
        out = (C.c_int * D)()
        st = None if starts is None else (C.c_int * D)(*[int(s) for s in starts])
        _check(lib().pv_run_subspace(self._p, C.byref(prm), int(D), st, C.byref(res), hist, n, out))
        rows = []
        for h in hist[:res.iterations]:
            rows.append(dict(lam=np.array(h.lambda_[:D]), E=np.array(h.energy[:D]), rho=np.array(h.rho[:D]),
                             s_norm=np.array(h.s_norm[:D]), lam_star=np.array(h.lambda_star[:D]),
                             bound=h.bound, eta=h.eta_res, eta_psi=h.eta_psi, seconds=h.seconds,
                             retries=h.retries, cap_bound=bool(h.cap_bound), max_rank=h.max_rank,
                             stop=bool(h.stopped)))
        return dict(energy=res.energy, lam=res.lambda_, rho=res.rho, bound=res.bound,
                    iterations=res.iterations, converged=bool(res.converged)), rows, list(out)

    def run_subspace_joint(self, D, start=-1, **kw):
        """Algorithm 4 with the columns held jointly (pv_run_subspace_joint).  Returns
        (result dict of column 1, rows, handle of the final joint MPS)."""
        if not 1 <= D <= SUBSPACE_MAX_D:
            raise ValueError(f"D must be in 1..{SUBSPACE_MAX_D}")
        kw.setdefault("max_iter", 20)
        n = max(kw["max_iter"], 1)
        prm = make_params(**kw)
        res = Result()
        hist = (SubspaceIter * n)()
        out = C.c_int()
        _check(lib().pv_run_subspace_joint(self._p, C.byref(prm), int(D), int(start), C.byref(res), hist, n,
                                           C.byref(out)))
        rows = []
        for h in hist[:res.iterations]:
            rows.append(dict(lam=np.array(h.lambda_[:D]), E=np.array(h.energy[:D]), rho=np.array(h.rho[:D]),
                             s_norm=np.array(h.s_norm[:D]), lam_star=np.array(h.lambda_star[:D]),
                             bound=h.bound, eta=h.eta_res, eta_psi=h.eta_psi, seconds=h.seconds,
                             retries=h.retries, cap_bound=bool(h.cap_bound), max_rank=h.max_rank,
                             stop=bool(h.stopped)))
        return dict(energy=res.energy, lam=res.lambda_, rho=res.rho, bound=res.bound,
                    iterations=res.iterations, converged=bool(res.converged)), rows, out.value

    def sym_eig(self, A, method, nvec=None):
        A = _f64(np.asfortranarray(A))
        n = A.shape[0]
        w = np.zeros(n)
        V = np.zeros((n, n), order="F")
        Vp = V.ctypes.data_as(C.POINTER(C.c_double))
        if nvec is None:
            _check(lib().pv_sym_eig(self._p, n, _dp(A.ravel(order="F")), _dp(w), Vp, int(method)))
        else:
            if method != 1:
                raise ValueError("a partial eigenvector set needs method 1")
            _check(lib().pv_sym_eig_top(self._p, n, _dp(A.ravel(order="F")), _dp(w), Vp, int(nvec)))
        return w, V

    def sym_eig_noalloc(self, n, A_ptr, w_ptr, V_ptr):
        """pv_sym_eig_noalloc on device buffers given as integer addresses (the caller's)."""
        _check(lib().pv_sym_eig_noalloc(self._p, int(n), C.c_void_p(A_ptr), C.c_void_p(w_ptr), C.c_void_p(V_ptr)))

    def gemm(self, A, B, Cin=None, ta=False, tb=False, alpha=1.0, beta=0.0, precision=0):
        """alpha op(A) op(B) + beta C on the device (column-major copies of the operands)."""
        A = _f64(np.asfortranarray(A))
        B = _f64(np.asfortranarray(B))
        M = A.shape[1] if ta else A.shape[0]
        K = A.shape[0] if ta else A.shape[1]
        N = B.shape[0] if tb else B.shape[1]
        if (B.shape[1] if tb else B.shape[0]) != K:
            raise ValueError("inner dimensions differ")
        Cm = np.zeros((M, N), order="F") if Cin is None else np.array(Cin, dtype=np.float64, order="F", copy=True)
        _check(lib().pv_gemm(self._p, M, N, K, _dp(A.ravel(order="F")), A.shape[0], int(bool(ta)),
                             _dp(B.ravel(order="F")), B.shape[0], int(bool(tb)),
                             _dp(Cm), M, float(alpha), float(beta), int(precision)))
        return Cm

    def mfma_f64_rate(self):
        """Attainable float64 MFMA rate of the device in TFLOP/s (pv_mfma_f64_rate)."""
        r = C.c_double(0.0)
        _check(lib().pv_mfma_f64_rate(self._p, C.byref(r)))
        return r.value

    def cholesky(self, A):
        A = _f64(np.asfortranarray(A))
        n = A.shape[0]
        W = np.zeros((n, n), order="F")
        _check(lib().pv_cholesky(self._p, n, _dp(A.ravel(order="F")), W.ctypes.data_as(C.POINTER(C.c_double))))
        return W

    def timers(self):
        n = 14
        ms, fl, by = np.zeros(n), np.zeros(n), np.zeros(n)
        calls = np.zeros(n, np.int32)
        _check(lib().pv_timers(self._p, n, _dp(ms), _dp(fl), _dp(by), _ip(calls)))
        return {lib().pv_timer_name(i).decode(): dict(ms=ms[i], flops=fl[i], bytes=by[i], calls=int(calls[i]))
                for i in range(n)}

    def timers_reset(self):
        _check(lib().pv_timers_reset(self._p))

    def set_timed_classes(self, names=None):
        """Time only the named kernel classes (None: all of them)."""
        if names is None:
            mask = 0xFFFFFFFF
        else:
            index = {lib().pv_timer_name(i).decode(): i for i in range(32) if lib().pv_timer_name(i)}
            unknown = set(names) - set(index)
            if unknown:
                raise ValueError(f"unknown kernel classes {sorted(unknown)}")
            mask = sum(1 << index[n] for n in set(names))
        _check(lib().pv_set_timer_mask(self._p, mask))

    def set_timer_sampling(self, names=None, every=1):
        """Time the named classes on a pseudo-random one-in-`every` subset of their launches
        (pv_set_timer_sampling); None or every = 1: every launch."""
        index = {lib().pv_timer_name(i).decode(): i for i in range(32) if lib().pv_timer_name(i)}
        names = names or []
        unknown = set(names) - set(index)
        if unknown:
            raise ValueError(f"unknown kernel classes {sorted(unknown)}")
        mask = sum(1 << index[n] for n in set(names))
        _check(lib().pv_set_timer_sampling(self._p, mask, int(every)))
