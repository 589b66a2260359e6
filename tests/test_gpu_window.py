"""Quantum-number block-sparse two-site product (the product inside the local
solves, eq. mat_vec) against the oracle's dense einsum definition.

Operands carry the charge structure of a real iterate: environments
E[K][bra][ket] are random where q(bra) - q(ket) equals the channel charge of K
and zero elsewhere, x is random on its allowed blocks.  Windows with and
without the coefficient block of the MPO are covered, and the three forms of the
product: both environments precontracted with their site tensors (default), only
the left one, and none (L x, then both site tensors as sparse mixes).  Tolerances
relative to
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
    ctx, mpo, labels = small
    _window_case(ctx, mpo, labels, b, prec)


@pytest.fixture(scope="module")
def small_modes(small):
    """Contexts that force the two ways the light rows of a channel mix read their
    inputs: every tile staged in LDS (1), or every entry read directly (2)."""
    from paper_2505_23429_amd.api import Context

    _, mpo, labels = small
    out = {}
    for mode in (1, 2):
        c = Context(chi=48, mix_stage=mode)
        c.set_mpo(mpo)
        out[mode] = c
    return out, mpo, labels


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("b", [1, 3, 5])
def test_window_product_staging_modes(small_modes, b, prec, mode):
    ctxs, mpo, labels = small_modes
    _window_case(ctxs[mode], mpo, labels, b, prec)


@pytest.fixture(scope="module")
def small_forms(small):
    """Contexts with the other two forms of the product: only the left operator
    precontracted (1), and none (0: L x, both site tensors as sparse mixes)."""
    from paper_2505_23429_amd.api import Context

    _, mpo, labels = small
    out = {}
    for form in (0, 1):
        c = Context(chi=48, precontract=form)
        c.set_mpo(mpo)
        out[form] = c
    return out, mpo, labels


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("b", [1, 3, 4, 5])
def test_window_product_other_forms(small_forms, b, prec, form):
    ctxs, mpo, labels = small_forms
    _window_case(ctxs[form], mpo, labels, b, prec)


def _window_case(ctx, mpo, labels, b, prec):
    import torch
    from paper_2505_23429_amd.api import window_apply

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


def _qn_env_dev(gen, lab, chan):
    """Device version of _qn_env (seeded torch generator on the GPU): for the
    full-size cases, whose environments are too large to draw on the host."""
    import torch

    r, rp, R = len(lab), _pad(len(lab)), len(chan)
    labt = torch.as_tensor(np.asarray(lab), device="cuda")
    diff = labt[:, None, :] - labt[None, :, :]
    E = torch.zeros((R, rp, rp), dtype=torch.float64, device="cuda")
    uniq, inv = np.unique(np.asarray(chan), axis=0, return_inverse=True)
    inv = np.asarray(inv).reshape(-1)
    for u, q in enumerate(uniq):
        ks = torch.as_tensor(np.nonzero(inv == u)[0], device="cuda")
        m = (diff == torch.as_tensor(q, device="cuda")).all(-1).to(torch.float64)
        blk = torch.randn((len(ks), r, r), generator=gen, dtype=torch.float64, device="cuda") / np.sqrt(r)
        E[ks, :r, :r] = blk * m[None]
    return E


# full-size windows: (L, integrals seed, chi, MPS seed, window, precision)
# (windows right of the coefficient-block site have heavy output rows whose operator
# entries split into shared inputs and private ones)
FULL = [(32, 1003, 512, 1004, 13, "f32"), (32, 1003, 512, 1004, 15, "f32"), (32, 1003, 512, 1004, 20, "f32"),
        (16, 1002, 256, 1003, 7, "f64"), (16, 1002, 256, 1003, 10, "f64"), (24, 1004, 1024, 1005, 12, "bf16")]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("L,seed,chi,mseed,b,prec", FULL)
def test_window_product_full_size_sampled(L, seed, chi, mseed, b, prec):
    """Workload sizes (L = 32, chi = 512 FP32; L = 16, chi = 256 FP64; L = 24,
    chi = 1024 bfloat16) with the real channel counts, windows without and with
    the coefficient block on either site: sampled outputs against the oracle."""
    import torch
    from paper_2505_23429_amd.api import Context, window_apply
    from paper_2505_23429_amd.mpo import build_mpo

    h, B = S.integrals(L, L, seed)
    mpo = build_mpo(h, B)
    _, labels = S.random_mps(L, L, 0, chi, mseed)
    ql, qr = np.asarray(labels[b]), np.asarray(labels[b + 2])
    rl, rr = len(ql), len(qr)
    print(f"L={L} chi={chi} window ({b},{b + 1}) {prec} rl={rl} rr={rr} "
          f"R={mpo.R[b]},{mpo.R[b + 1]},{mpo.R[b + 2]}", flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7 + b)
    Ld = _qn_env_dev(gen, ql, mpo.chan_q[b])
    Rd = _qn_env_dev(gen, qr, mpo.chan_q[b + 2])
    rng = np.random.default_rng(7 + b)
    x = _qn_x(rng, ql, qr)
    rows = [0, rl // 2, rl - 1]
    cols = [3, rr // 2 + 1, rr - 1]
    # the rows the oracle needs, and the operands it sees (rounded as the device rounds them)
    Lrows = [Ld[:, i, :rl].cpu().numpy() for i in rows]
    Rrows = [Rd[:, j, :rr].cpu().numpy() for j in cols]
    xo = x
    if prec == "bf16":
        to_bf = lambda a: torch.from_numpy(a).float().bfloat16().double().numpy()
        Lrows, Rrows, xo = [to_bf(a) for a in Lrows], [to_bf(a) for a in Rrows], to_bf(x)
    ctx = Context(chi=chi)
    ctx.set_mpo(mpo)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    y = window_apply(ctx, b, ql, qr, Ld, Rd, xd, prec).cpu().numpy()
    del Ld, Rd, xd
    torch.cuda.empty_cache()
    print("device product done", flush=True)
    W1 = (mpo.A[b], mpo.B[b], mpo.ops[b])
    W2 = (mpo.A[b + 1], mpo.B[b + 1], mpo.ops[b + 1])
    ys = C.heff_rows(Lrows, xo[:rl, :, :, :rr], W1, W2, mpo.R[b + 1], mpo.R[b + 2], Rrows)
    scale = np.abs(ys).max()
    assert scale > 0
    for ii, i in enumerate(rows):
        for jj, j in enumerate(cols):
            assert np.abs(y[i, :, :, j] - ys[ii, jj]).max() <= TOL[prec] * scale, (i, j)
    # structurally zero outputs are exactly zero
    sc = np.asarray(S.SITE_CHARGES)
    for i in rows:
        for j in cols:
            for u in range(4):
                for v in range(4):
                    if not np.all(ql[i] + sc[u] + sc[v] == qr[j]):
                        assert y[i, u, v, j] == 0.0
    ctx.close()
