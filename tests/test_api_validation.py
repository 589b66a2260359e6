"""The Python binding validates every device operand before its pointer crosses
the C ABI: a tensor of the wrong shape, dtype or layout raises ValueError
before any device call (no context or GPU is touched: ctx is None here)."""
import numpy as np
import pytest
import torch

from paper_2505_23429_amd import api


def _w(R_in, R_out, nnz=3, seed=0):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, R_in, nnz), rng.integers(0, R_out, nnz), rng.standard_normal((nnz, 4, 4)))


def test_heff_apply_rejects_bad_operands():
    L = torch.zeros((3, 32, 32), dtype=torch.float64)
    R = torch.zeros((2, 64, 64), dtype=torch.float64)
    x = torch.zeros((32, 4, 4, 64), dtype=torch.float64)
    W1, W2 = _w(3, 5), _w(5, 2)
    with pytest.raises(ValueError, match="shape"):
        api.heff_apply_rb(None, "f64", L, W1, W2, R, torch.zeros((32, 4, 4, 32), dtype=torch.float64), 5)
    with pytest.raises(ValueError, match="dtype"):
        api.heff_apply_rb(None, "f64", L.float(), W1, W2, R, x, 5)
    with pytest.raises(ValueError, match="dtype"):
        api.heff_apply_rb(None, "bf16", L, W1, W2, R, x, 5)
    with pytest.raises(ValueError, match="contiguous"):
        api.heff_apply_rb(None, "f64", L.transpose(1, 2), W1, W2, R, x, 5)
    with pytest.raises(ValueError, match="multiple of 32"):
        api.heff_apply_rb(None, "f64", torch.zeros((3, 30, 30), dtype=torch.float64), W1, W2, R,
                          torch.zeros((30, 4, 4, 64), dtype=torch.float64), 5)
    with pytest.raises(ValueError, match="channel index"):
        api.heff_apply_rb(None, "f64", L, _w(4, 5), W2, R, x, 5)
    with pytest.raises(ValueError, match="device"):
        api.heff_apply_rb(None, "f64", L, W1, W2, R, x, 5)
    with pytest.raises(ValueError, match="precision"):
        api.heff_apply_rb(None, "f16", L, W1, W2, R, x, 5)


def test_window_apply_rejects_bad_operands():
    ql = np.zeros((20, 2), dtype=np.int32)
    qr = np.zeros((40, 2), dtype=np.int32)
    L = torch.zeros((7, 32, 32), dtype=torch.float64)
    R = torch.zeros((9, 64, 64), dtype=torch.float64)
    x = torch.zeros((32, 4, 4, 64), dtype=torch.float64)
    with pytest.raises(ValueError, match="shape"):
        api.window_apply(None, 0, ql, qr, L, R, torch.zeros((20, 4, 4, 40), dtype=torch.float64))
    with pytest.raises(ValueError, match="shape"):
        api.window_apply(None, 0, ql, qr, torch.zeros((7, 20, 20), dtype=torch.float64), R, x)
    with pytest.raises(ValueError, match="dtype"):
        api.window_apply(None, 0, ql, qr, L, R.float(), x)
    with pytest.raises(ValueError, match="label"):
        api.window_apply(None, 0, ql[:, 0], qr, L, R, x)
    with pytest.raises(ValueError, match="device"):
        api.window_apply(None, 0, ql, qr, L, R, x)


def test_env_update_rejects_bad_operands():
    W = _w(3, 4)
    Ub = torch.zeros((32, 4, 64), dtype=torch.float64)
    Uk = torch.zeros((32, 4, 64), dtype=torch.float64)
    with pytest.raises(ValueError, match="shape"):
        api.env_update(None, 0, torch.zeros((3, 32, 64), dtype=torch.float64), Ub, Uk, W, 3, 4)
    with pytest.raises(ValueError, match="shape"):
        api.env_update(None, 1, torch.zeros((3, 32, 32), dtype=torch.float64), Ub, Uk, W, 3, 4)
    with pytest.raises(ValueError, match="side"):
        api.env_update(None, 2, torch.zeros((3, 32, 32), dtype=torch.float64), Ub, Uk, W, 3, 4)
    with pytest.raises(ValueError, match="device"):
        api.env_update(None, 0, torch.zeros((3, 32, 32), dtype=torch.float64), Ub, Uk, W, 3, 4)


def test_gemm_rejects_undersized_operands():
    M, N, K, batch, kin = 40, 24, 64, 2, 32
    strides = (M * K, K, kin, 1, K * N, kin * N, N, 1, M * N, N)
    A = torch.zeros(batch * M * K, dtype=torch.float64)
    B = torch.zeros(batch * K * N, dtype=torch.float64)
    Cm = torch.zeros(batch * M * N, dtype=torch.float64)
    with pytest.raises(ValueError, match="elements"):
        api.gemm(None, "f64", M, N, K, batch, kin, strides, 1, 1, A[:-1], B, Cm)
    with pytest.raises(ValueError, match="elements"):
        api.gemm(None, "f64", M, N, K, batch, kin, strides, 1, 1, A, B, Cm[: M * N])
    with pytest.raises(ValueError, match="dtype"):
        api.gemm(None, "bf16", M, N, K, batch, kin, strides, 1, 1, A, B, Cm)
    with pytest.raises(ValueError, match="kin"):
        api.gemm(None, "f64", M, N, K + 1, batch, kin, strides, 1, 1, A, B, Cm)
    with pytest.raises(ValueError, match="device"):
        api.gemm(None, "f64", M, N, K, batch, kin, strides, 1, 1, A, B, Cm)


def test_heff_energy_grad_rejects_bad_operands():
    L = torch.zeros((3, 32, 32), dtype=torch.float64)
    R = torch.zeros((2, 32, 32), dtype=torch.float64)
    x = torch.zeros((32, 4, 4, 32), dtype=torch.float32)
    with pytest.raises(ValueError, match="dtype"):
        api.heff_energy_grad(None, L, _w(3, 5), _w(5, 2), R, x, 5)
    W2 = (np.array([0, 4]), np.array([1, 2]), np.zeros((2, 4, 4)))  # right channel 2 >= RC = 2
    with pytest.raises(ValueError, match="channel index"):
        api.heff_energy_grad(None, L, _w(3, 5), W2, R, x.double(), 5)


@pytest.mark.parametrize("kw", [{"precontract": 3}, {"precontract": -1}, {"functional": "min"}, {"svd_blocked": 5}])
def test_context_rejects_bad_options_before_create(kw):
    """Options the binding can check itself are refused before tt_create runs, so no
    device is touched (the library is only loaded)."""
    with pytest.raises(ValueError):
        api.Context(chi=16, **kw)
