"""Kernel-level parity of the HIP path against the oracle's einsum definitions.

Sizes span several 128x128 GEMM tiles with ragged tails (bond dimensions that
are multiples of 32 but not of 128).  Tolerances: relative to max|y|,
1e-12 in FP64, 1e-5 in FP32 (FP32 accumulation over K <= 10^5 terms), 2e-2
for BF16 operands (unit roundoff 2^-8 on L, R, x and the rounded intermediate).
"""
import numpy as np
import pytest

import seeded_inputs as S
from oracle import contract as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_23429_amd.api import Context

    return Context(chi=64)


def _dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _case(rl, rr, RA, RB, RC, seed, nnz=3):
    Lenv, W1, W2, Renv, x = S.heff_operands(rl, rr, RA, RB, RC, seed, nnz)
    ref = C.heff_apply(Lenv.transpose(1, 0, 2), C.dense_core(*W1, RA, RB), C.dense_core(*W2, RB, RC),
                       Renv.transpose(1, 0, 2), x)
    return Lenv, W1, W2, Renv, x, ref


@pytest.mark.parametrize("rl,rr,RA,RB,RC", [(32, 32, 1, 3, 2), (64, 96, 7, 9, 5), (160, 96, 13, 17, 11)])
def test_heff_f64(ctx, rl, rr, RA, RB, RC):
    import torch
    from paper_2505_23429_amd.api import heff_apply_rb

    Lenv, W1, W2, Renv, x, ref = _case(rl, rr, RA, RB, RC, seed=rl + rr + RA)
    y = heff_apply_rb(ctx, "f64", _dev(Lenv), W1, W2, _dev(Renv), _dev(x), RB)
    torch.cuda.synchronize()
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err


@pytest.mark.parametrize("rl,rr,RA,RB,RC", [(64, 96, 7, 9, 5), (128, 160, 11, 13, 9)])
def test_heff_f32(ctx, rl, rr, RA, RB, RC):
    import torch
    from paper_2505_23429_amd.api import heff_apply_rb

    Lenv, W1, W2, Renv, x, ref = _case(rl, rr, RA, RB, RC, seed=7 * rl + rr)
    y = heff_apply_rb(ctx, "f32", _dev(Lenv, torch.float32), W1, W2, _dev(Renv, torch.float32),
                      _dev(x, torch.float32), RB)
    err = np.abs(y.double().cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-5, err


@pytest.mark.parametrize("rl,rr,RA,RB,RC", [(64, 96, 7, 9, 5), (128, 160, 11, 13, 9)])
def test_heff_bf16(ctx, rl, rr, RA, RB, RC):
    import torch
    from paper_2505_23429_amd.api import heff_apply_rb

    Lenv, W1, W2, Renv, x, _ = _case(rl, rr, RA, RB, RC, seed=11 * rl + rr)
    Lb = _dev(Lenv, torch.bfloat16)
    Rb = _dev(Renv, torch.bfloat16)
    xb = _dev(x, torch.bfloat16)
    # the oracle sees the same bf16-rounded operands
    ref = C.heff_apply(Lb.double().cpu().numpy().transpose(1, 0, 2), C.dense_core(*W1, RA, RB),
                       C.dense_core(*W2, RB, RC), Rb.double().cpu().numpy().transpose(1, 0, 2),
                       xb.double().cpu().numpy())
    y = heff_apply_rb(ctx, "bf16", Lb, W1, W2, Rb, xb, RB)
    err = np.abs(y.double().cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 2e-2, err


@pytest.mark.parametrize("rb,rk,rb2,rk2", [(32, 64, 96, 64), (96, 96, 32, 64)])
def test_env_updates_f64(ctx, rb, rk, rb2, rk2):
    from paper_2505_23429_amd.api import env_update

    rng = np.random.default_rng(rb * 3 + rk2)
    RA, RB = 6, 8
    A, B, ops = S.random_sparse_mpo_core(RA, RB, 3, seed=int(rb2))
    W = C.dense_core(A, B, ops, RA, RB)
    Ubra = rng.standard_normal((rb, 4, rb2))
    Uket = rng.standard_normal((rk, 4, rk2))
    El = rng.standard_normal((RA, rb, rk))
    out = env_update(ctx, 0, _dev(El), _dev(Ubra), _dev(Uket), (A, B, ops), RA, RB)
    ref = C.env_left(El.transpose(1, 0, 2), Ubra, W, Uket).transpose(1, 0, 2)
    assert np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max() < 1e-12
    Er = rng.standard_normal((RB, rb2, rk2))
    out = env_update(ctx, 1, _dev(Er), _dev(Ubra), _dev(Uket), (A, B, ops), RA, RB)
    ref = C.env_right(Er.transpose(1, 0, 2), Ubra, W, Uket).transpose(1, 0, 2)
    assert np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max() < 1e-12


def test_heff_energy_gradients(ctx):
    from paper_2505_23429_amd.api import heff_energy_grad

    rl, rr, RA, RB, RC = 64, 32, 5, 7, 4
    Lenv, W1, W2, Renv, x = S.heff_operands(rl, rr, RA, RB, RC, seed=99, nnz_per_col=2)
    D1 = C.dense_core(*W1, RA, RB)
    D2 = C.dense_core(*W2, RB, RC)
    E, gx, gL, gW1, gW2, gR = C.heff_grads(Lenv.transpose(1, 0, 2), D1, D2, Renv.transpose(1, 0, 2), x)
    Eg, gxg, gLg, gRg, g1, g2 = heff_energy_grad(ctx, _dev(Lenv), W1, W2, _dev(Renv), _dev(x), RB)
    sc = max(1.0, abs(E))
    assert abs(Eg - E) < 1e-11 * sc
    assert np.abs(gxg.cpu().numpy() - gx).max() < 1e-11 * np.abs(gx).max()
    assert np.abs(gLg.cpu().numpy() - gL.transpose(1, 0, 2)).max() < 1e-11 * np.abs(gL).max()
    assert np.abs(gRg.cpu().numpy() - gR.transpose(1, 0, 2)).max() < 1e-11 * np.abs(gR).max()
    # each entry's gradient is the dense gradient at (A, :, :, B)
    ref1 = gW1[W1[0], :, :, W1[1]]
    ref2 = gW2[W2[0], :, :, W2[1]]
    assert np.abs(g1 - ref1).max() < 1e-11 * np.abs(ref1).max()
    assert np.abs(g2 - ref2).max() < 1e-11 * np.abs(ref2).max()


@pytest.mark.timeout(600)
def test_heff_full_size_sampled_outputs(ctx):
    """Middle window of the L=32, chi=512 workload (FP32 product, real MPO
    channel counts and sparsity): sampled outputs against the oracle."""
    import torch
    from paper_2505_23429_amd.api import heff_apply_rb
    from paper_2505_23429_amd.mpo import build_mpo

    L = 32
    h, B = S.integrals(L, L, 1003)
    mpo = build_mpo(h, B)
    b = L // 2 - 3  # window (13, 14): no coefficient block inside
    r = 512
    RA, RB, RC = mpo.R[b], mpo.R[b + 1], mpo.R[b + 2]
    rng = np.random.default_rng(5)
    Lenv = (rng.standard_normal((RA, r, r)) / np.sqrt(r)).astype(np.float32)
    Renv = (rng.standard_normal((RC, r, r)) / np.sqrt(r)).astype(np.float32)
    x = rng.standard_normal((r, 4, 4, r)).astype(np.float32)
    W1 = (mpo.A[b], mpo.B[b], mpo.ops[b])
    W2 = (mpo.A[b + 1], mpo.B[b + 1], mpo.ops[b + 1])
    y = heff_apply_rb(ctx, "f32", _dev(Lenv), W1, W2, _dev(Renv), _dev(x), RB).double().cpu().numpy()
    rows = [0, 511]
    cols = [3, 400]
    ys = C.heff_rows([Lenv[:, i, :].astype(np.float64) for i in rows], x.astype(np.float64),
                     (W1[0], W1[1], W1[2]), (W2[0], W2[1], W2[2]), RB, RC,
                     [Renv[:, j, :].astype(np.float64) for j in cols])
    scale = np.abs(ys).max()
    for ii, i in enumerate(rows):
        for jj, j in enumerate(cols):
            assert np.abs(y[i, :, :, j] - ys[ii, jj]).max() < 1e-4 * scale
    del y
    torch.cuda.empty_cache()
