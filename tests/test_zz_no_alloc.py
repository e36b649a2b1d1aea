"""The allocation-free dense SPD entry point (pdipc_dense_spd_noalloc) against
the allocating one (pdipc_debug_dense) through the C ABI: the same kernels on
the same inputs, two calls in a row (the second smaller, so that it runs on
what the first left in the shared scratch array), both precisions; plus the
size limit and the pivot report."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    return G @ G.T / n + 0.5 * np.eye(n), rng.standard_normal((n, 3))


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_allocating_entry_point(precision):
    from paper_2312_02999_amd import dense_spd, dense_spd_noalloc
    for n, seed in ((1000, 11), (130, 12)):       # second call smaller
        A, b = _spd(n, seed)
        At, bt = _t(A), _t(b)
        x_ref, inv_ref = dense_spd(At, bt, inverse=True, precision=precision)
        x, inv, info = dense_spd_noalloc(At, bt, inverse=True, precision=precision)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        xr, ir = x_ref.cpu().numpy(), inv_ref.cpu().numpy()
        xg, ig = x.cpu().numpy(), inv.cpu().numpy()
        # same kernels and inputs: the results agree to rounding (in fact bitwise)
        scale_x, scale_i = np.abs(xr).max(), np.abs(ir).max()
        print(f"noalloc n={n} precision={precision}: max |dx| {np.abs(xg - xr).max() / scale_x:.2e} "
              f"max |dinv| {np.abs(ig - ir).max() / scale_i:.2e}")
        assert np.abs(xg - xr).max() <= 1e-12 * scale_x
        assert np.abs(ig - ir).max() <= 1e-12 * scale_i
        # and both solve the system (FP64 to 1e-10, FP32 to 1e-3)
        tol = 1e-10 if precision == 0 else 1e-3
        xs = np.linalg.solve(A, b)
        assert np.abs(xg - xs).max() <= tol * max(1.0, np.abs(xs).max())
        # the input matrix is not modified
        assert np.array_equal(At.cpu().numpy(), A)


def test_noalloc_single_rhs_and_no_outputs():
    from paper_2312_02999_amd import dense_spd_noalloc
    A, b = _spd(257, 13)
    x, inv, info = dense_spd_noalloc(_t(A), _t(b[:, 0]))
    torch.cuda.synchronize()
    assert inv is None and int(info.item()) == 0
    xs = np.linalg.solve(A, b[:, 0])
    assert np.abs(x.cpu().numpy() - xs).max() <= 1e-10 * max(1.0, np.abs(xs).max())
    # factor only: info alone
    _, _, info = dense_spd_noalloc(_t(A))
    torch.cuda.synchronize()
    assert int(info.item()) == 0


def test_noalloc_reports_non_positive_pivot():
    from paper_2312_02999_amd import dense_spd_noalloc
    A = np.eye(70)
    A[66, 66] = -1.0
    _, _, info = dense_spd_noalloc(_t(A), _t(np.ones((70, 1))))
    torch.cuda.synchronize()
    assert int(info.item()) == 67


def test_noalloc_rejects_order_beyond_its_array():
    from paper_2312_02999_amd import PdipcError, dense_spd_noalloc
    A = torch.eye(1025, dtype=torch.float64, device=DEV)
    with pytest.raises(PdipcError) as ei:
        dense_spd_noalloc(A, torch.ones(1025, 1, dtype=torch.float64, device=DEV))
    assert "1024" in str(ei.value)
