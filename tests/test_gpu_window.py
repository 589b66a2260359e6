"""Quantum-number block-sparse two-site product (the product inside the local
solves, eq. mat_vec) against the oracle's dense einsum definition.

Operands carry the charge structure of a real iterate: environments
E[K][bra][ket] are random where q(bra) - q(ket) equals the channel charge of K
and zero elsewhere, x is random on its allowed blocks.  Windows with and
without the coefficient block of the MPO are covered.  Tolerances relative to
max|y|: 1e-12 (FP64), 1e-5 (FP32), 2e-2 (bfloat16-rounded operands).
"""
import numpy as np
import pytest

import seeded_inputs as S
from oracle import contract as C

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}


def _pad(r):
    return ((r + 31) // 32) * 32


def _qn_env(rng, lab, chan, dtype=np.float64):
    """Random environment [R][rp][rp] (zero padded), non-zero only where
    q(bra) - q(ket) equals the channel charge."""
    r, rp, R = len(lab), _pad(len(lab)), len(chan)
    diff = lab[:, None, :] - lab[None, :, :]
    E = np.zeros((R, rp, rp), dtype=dtype)
    uniq, inv = np.unique(np.asarray(chan), axis=0, return_inverse=True)
    inv = np.asarray(inv).reshape(-1)
    for u, q in enumerate(uniq):
        ks = np.nonzero(inv == u)[0]
        m = np.all(diff == q[None, None, :], axis=-1)
        blk = rng.standard_normal((len(ks), r, r)).astype(dtype) / np.sqrt(r)
        E[ks, :r, :r] = blk * m[None]
    return E


def _qn_x(rng, ql, qr):
    rl, rr = len(ql), len(qr)
    sc = np.asarray(S.SITE_CHARGES)
    tot = ql[:, None, None, :] + sc[None, :, None, :] + sc[None, None, :, :]
    allowed = np.all(tot[:, :, :, None, :] == qr[None, None, None, :, :], axis=-1)
    x = np.zeros((_pad(rl), 4, 4, _pad(rr)))
    x[:rl, :, :, :rr] = rng.standard_normal((rl, 4, 4, rr)) * allowed
    return x


@pytest.fixture(scope="module")
def small():
    from paper_2505_23429_amd.api import Context
    from paper_2505_23429_amd.mpo import build_mpo

    L = 8
    h, B = S.integrals(L, L, 1008)
    mpo = build_mpo(h, B)
    _, labels = S.random_mps(L, L, 0, 48, 31)
    ctx = Context(chi=48)
    ctx.set_mpo(mpo)
    return ctx, mpo, labels


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("b", [1, 3, 4])
def test_window_product_matches_oracle(small, b, prec):
    import torch
    from paper_2505_23429_amd.api import window_apply

    ctx, mpo, labels = small
    ql, qr = np.asarray(labels[b]), np.asarray(labels[b + 2])
    rl, rr = len(ql), len(qr)
    rng = np.random.default_rng(100 + b)
    Lenv = _qn_env(rng, ql, mpo.chan_q[b])
    Renv = _qn_env(rng, qr, mpo.chan_q[b + 2])
    x = _qn_x(rng, ql, qr)
    if prec == "bf16":
        # the oracle sees the same bfloat16-rounded operands
        to_bf = lambda a: torch.from_numpy(a).float().bfloat16().double().numpy()
        Lr, Rr, xr = to_bf(Lenv), to_bf(Renv), to_bf(x)
    else:
        Lr, Rr, xr = Lenv, Renv, x
    W1 = C.dense_core(mpo.A[b], mpo.B[b], mpo.ops[b], mpo.R[b], mpo.R[b + 1])
    W2 = C.dense_core(mpo.A[b + 1], mpo.B[b + 1], mpo.ops[b + 1], mpo.R[b + 1], mpo.R[b + 2])
    ref = C.heff_apply(Lr[:, :rl, :rl].transpose(1, 0, 2), W1, W2, Rr[:, :rr, :rr].transpose(1, 0, 2),
                       xr[:rl, :, :, :rr])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    y = window_apply(ctx, b, ql, qr, dev(Lenv), dev(Renv), dev(x), prec).cpu().numpy()
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(y[:rl, :, :, :rr] - ref).max() <= TOL[prec] * scale
    # padding rows and columns stay zero
    assert np.all(y[rl:] == 0) and np.all(y[:, :, :, rr:] == 0)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("b", [13, 15])
def test_window_product_full_size_sampled(b):
    """L = 32, chi = 512 workload (FP32 product, real channel counts, window
    (13, 14) and the coefficient-block window (15, 16)): sampled outputs."""
    import torch
    from paper_2505_23429_amd.api import Context, window_apply
    from paper_2505_23429_amd.mpo import build_mpo

    L = 32
    h, B = S.integrals(L, L, 1003)
    mpo = build_mpo(h, B)
    _, labels = S.random_mps(L, L, 0, 512, 1004)
    ql, qr = np.asarray(labels[b]), np.asarray(labels[b + 2])
    rl, rr = len(ql), len(qr)
    print(f"window ({b},{b + 1}) rl={rl} rr={rr} R={mpo.R[b]},{mpo.R[b + 1]},{mpo.R[b + 2]}", flush=True)
    rng = np.random.default_rng(7 + b)
    Lenv = _qn_env(rng, ql, mpo.chan_q[b])
    Renv = _qn_env(rng, qr, mpo.chan_q[b + 2])
    x = _qn_x(rng, ql, qr)
    ctx = Context(chi=512)
    ctx.set_mpo(mpo)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Ld, Rd, xd = dev(Lenv), dev(Renv), dev(x)
    y = window_apply(ctx, b, ql, qr, Ld, Rd, xd, "f32").cpu().numpy()
    del Ld, Rd, xd
    torch.cuda.empty_cache()
    print("device product done", flush=True)
    rows = [0, rl // 2, rl - 1]
    cols = [3, rr // 2 + 1, rr - 1]
    W1 = (mpo.A[b], mpo.B[b], mpo.ops[b])
    W2 = (mpo.A[b + 1], mpo.B[b + 1], mpo.ops[b + 1])
    ys = C.heff_rows([Lenv[:, i, :rl] for i in rows], x[:rl, :, :, :rr], W1, W2, mpo.R[b + 1], mpo.R[b + 2],
                     [Renv[:, j, :rr] for j in cols])
    scale = np.abs(ys).max()
    assert scale > 0
    for ii, i in enumerate(rows):
        for jj, j in enumerate(cols):
            assert np.abs(y[i, :, :, j] - ys[ii, jj]).max() <= TOL["f32"] * scale, (i, j)
    # structurally zero outputs are exactly zero
    sc = np.asarray(S.SITE_CHARGES)
    for i in rows:
        for j in cols:
            for u in range(4):
                for v in range(4):
                    if not np.all(ql[i] + sc[u] + sc[v] == qr[j]):
                        assert y[i, u, v, j] == 0.0
    ctx.close()
