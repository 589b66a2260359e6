"""The strided MFMA GEMM against numpy for every operand layout, a two-level K
index and ragged tiles (FP64 exact to 1e-13, FP32 1e-6, BF16 operands 1e-2)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_23429_amd.api import Context

    return Context()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("akc", [True, False])
@pytest.mark.parametrize("bnc", [True, False])
def test_gemm_layouts(ctx, prec, akc, bnc):
    import torch
    from paper_2505_23429_amd.api import gemm

    rng = np.random.default_rng(3)
    batch, M, N, kb, kin = 2, 150, 70, 3, 32
    K = kb * kin
    A = rng.standard_normal((batch, M, K))
    B = rng.standard_normal((batch, K, N))
    ref = A @ B
    # store A as [b][kb][m][kin] (k-contiguous) or [b][kb][kin][m] (m-contiguous)
    if akc:
        As = A.reshape(batch, M, kb, kin).transpose(0, 2, 1, 3).copy()
        sA = (kb * M * kin, kin, M * kin, 1)
    else:
        As = A.reshape(batch, M, kb, kin).transpose(0, 2, 3, 1).copy()
        sA = (kb * M * kin, 1, M * kin, M)
    if bnc:
        Bs = B.reshape(batch, kb, kin, N).copy()
        sB = (kb * kin * N, kin * N, N, 1)
    else:
        Bs = B.reshape(batch, kb, kin, N).transpose(0, 1, 3, 2).copy()
        sB = (kb * kin * N, kin * N, 1, kin)
    dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[prec]
    Ad = torch.from_numpy(As).to(dt).cuda()
    Bd = torch.from_numpy(Bs).to(dt).cuda()
    Cd = torch.zeros((batch, M, N), dtype=torch.float64 if prec == "f64" else torch.float32).cuda()
    strides = (*sA, *sB, M * N, N)
    gemm(ctx, prec, M, N, K, batch, kin, strides, akc, bnc, Ad, Bd, Cd)
    if prec == "bf16":
        Ar = Ad.double().cpu().numpy()
        Br = Bd.double().cpu().numpy()
        if akc:
            A2 = Ar.transpose(0, 2, 1, 3).reshape(batch, M, K)
        else:
            A2 = Ar.transpose(0, 3, 1, 2).reshape(batch, M, K)
        B2 = (Br if bnc else Br.transpose(0, 1, 3, 2)).reshape(batch, K, N)
        ref = A2 @ B2
    tol = {"f64": 1e-13, "f32": 1e-6, "bf16": 1e-5}[prec]
    err = np.abs(Cd.double().cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < tol, err
