"""The no-allocation entry point (tt_heff_apply_dev_noalloc) against the allocating one
(tt_heff_apply_dev), called through the C ABI: two calls in a row, the second smaller,
in FP64 and FP32; the same kernels on the same operands give the same bits.  Sizes
beyond the fixed scratch are refused before any device work."""
import ctypes as C

import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_23429_amd.api import Context

    c = Context(chi=64)
    yield c
    c.close()


def _operands(rl, rr, RA, RB, RC, seed, dtype):
    import torch

    Lenv, W1, W2, Renv, x = S.heff_operands(rl, rr, RA, RB, RC, seed, 3)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()
    return dev(Lenv), W1, W2, dev(Renv), dev(x)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_equals_allocating_entry_point(ctx, prec):
    import torch
    from paper_2505_23429_amd.api import heff_apply_noalloc, heff_apply_rb

    dt = torch.float64 if prec == "f64" else torch.float32
    for (rl, rr, RA, RB, RC, seed) in [(96, 64, 13, 17, 11, 5), (32, 32, 3, 5, 2, 6)]:
        Lenv, W1, W2, Renv, x = _operands(rl, rr, RA, RB, RC, seed, dt)
        ref = heff_apply_rb(ctx, prec, Lenv, W1, W2, Renv, x, RB)
        y = torch.full_like(x, float("nan"))
        heff_apply_noalloc(ctx, prec, Lenv, W1, W2, Renv, x, RB, y)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), (prec, rl, rr, float((y - ref).abs().max()))


def test_noalloc_refuses_products_beyond_its_scratch(ctx):
    import torch
    from paper_2505_23429_amd import _lib
    from paper_2505_23429_amd.api import TTError, heff_apply_noalloc

    # 2 x (RA + RB) slabs of 256*16*256 doubles exceed the fixed scratch; tiny tensors
    # suffice because the size check comes before any device access
    rl = rr = 256
    RA = RB = RC = 40
    need = (max(RA, RC) + RB) * rl * 16 * rr * 8
    assert need > _lib.TT_NOALLOC_SCRATCH_BYTES
    Lenv = torch.zeros((RA, rl, rl), dtype=torch.float64, device="cuda")
    Renv = torch.zeros((RC, rr, rr), dtype=torch.float64, device="cuda")
    x = torch.zeros((rl, 4, 4, rr), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    W = (np.arange(RA), np.arange(RB), np.zeros((RA, 4, 4)))
    with pytest.raises(TTError) as e:
        heff_apply_noalloc(ctx, "f64", Lenv, W, W, Renv, x, RB, y)
    assert e.value.code == _lib.TT_EINVAL and "scratch" in str(e.value)
