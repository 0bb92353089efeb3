"""The allocation-free entry point pv_sym_eig_noalloc (the eigensolver on caller-owned
device buffers, its work area in a fixed device array) against pv_sym_eig with method 1
on the same matrices: two calls in a row, the second with a smaller matrix, and the
rejection of a matrix larger than the array holds."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

native = pytest.importorskip("paper_2604_16118_amd.native")


def _matrix(n, seed):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((n, n // 2)) * np.logspace(0, -6, n // 2)[None, :]
    a = b @ b.T + 1e-3 * rng.standard_normal((n, n))
    return (a + a.T) / 2


def test_noalloc_eigensolver_matches_sym_eig_on_two_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with native.Context(0) as ctx:
        for n, seed in ((500, 1), (150, 2)):
            print(f"# pv_sym_eig_noalloc n={n}", flush=True)
            A = _matrix(n, seed)
            w_ref, V_ref = ctx.sym_eig(A, 1)
            dA = torch.from_numpy(A.ravel(order="F").copy()).to("cuda")
            dw = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
            dV = torch.full((n * n,), float("nan"), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            ctx.sym_eig_noalloc(n, dA.data_ptr(), dw.data_ptr(), dV.data_ptr())
            w = dw.cpu().numpy()
            V = dV.cpu().numpy().reshape(n, n, order="F")
            an = np.abs(w_ref).max()
            assert np.all(np.isfinite(w)) and np.all(np.isfinite(V))
            assert np.abs(w - w_ref).max() <= 1e-13 * an
            assert np.abs(V - V_ref).max() <= 1e-11
            keep = np.abs(w) > 1e-12 * an
            res = A @ V[:, keep] - V[:, keep] * w[keep]
            assert np.abs(res).max() <= 1e-10 * an
            assert np.allclose(np.sort(w), np.linalg.eigvalsh(A), rtol=0, atol=1e-12 * an * n / 100)


def test_noalloc_eigensolver_rejects_an_order_beyond_its_array():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = 513
    with native.Context(0) as ctx:
        dA = torch.zeros(n * n, dtype=torch.float64, device="cuda")
        dw = torch.zeros(n, dtype=torch.float64, device="cuda")
        dV = torch.zeros(n * n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(native.PvError) as e:
            ctx.sym_eig_noalloc(n, dA.data_ptr(), dw.data_ptr(), dV.data_ptr())
        assert e.value.status == -1 and "512" in str(e.value)
