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


def test_noalloc_eigensolver_keeps_the_step_reduction_under_the_panel_setting():
    """pv_set_tridiag_steps(ctx, 0) sends the context's own eigensolves to the panel
    reduction, whose trailing GEMM updates allocate their split-K partials; the
    allocation-free call keeps the step reduction and its fixed work area (the same bits as
    without the setting) and leaves the context's setting in force for its own solves."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = 300
    A = _matrix(n, 3)
    with native.Context(0) as ctx:
        dA = torch.from_numpy(A.ravel(order="F").copy()).to("cuda")
        out = []
        for steps in (native.TRIDIAG_STEPS_DEFAULT, 0):
            print(f"# pv_sym_eig_noalloc n={n} with pv_set_tridiag_steps({steps})", flush=True)
            ctx.set_tridiag_steps(steps)
            dw = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
            dV = torch.full((n * n,), float("nan"), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            ctx.sym_eig_noalloc(n, dA.data_ptr(), dw.data_ptr(), dV.data_ptr())
            out.append((dw.cpu().numpy(), dV.cpu().numpy()))
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
        w_panel, _ = ctx.sym_eig(A, 1)  # the context's own solve, on the panels
        an = np.abs(out[0][0]).max()
        assert np.abs(w_panel - out[0][0]).max() <= 1e-12 * an
        ctx.set_tridiag_steps(native.TRIDIAG_STEPS_DEFAULT)
