"""The torch.autograd Functions over the library's hand-written backward.

* HeffEnergy (E = <x|H_eff|x>, tt_heff_energy_grad_dev): the gradient with
  respect to x, both environments and both MPO cores against central
  differences.  E is quadratic in x and linear in every other operand, so a
  central difference is exact up to rounding.
* MpoEnergy (E = <U|H(ops)|U>, tt_energy_mpo_grad) composed with the linear map
  h -> ops: dE/dh by autograd at L = 16, chi = 256 (the differentiation
  workload), against the oracle's one-particle density matrix (dE/dh_pq =
  gamma_pq for a fixed state) and against a second context built from h + d.
"""
import numpy as np
import pytest

import seeded_inputs as S
from oracle import density as D

pytestmark = pytest.mark.gpu


def test_heff_energy_function_against_central_differences():
    import torch
    from paper_2505_23429_amd.api import Context, make_heff_energy

    rl, rr, RA, RB, RC = 32, 64, 5, 7, 4
    Lenv, W1, W2, Renv, x = S.heff_operands(rl, rr, RA, RB, RC, seed=77, nnz_per_col=3)
    ctx = Context(chi=64)
    F = make_heff_energy(ctx, (W1[0], W1[1]), (W2[0], W2[1]), RB)
    dev = torch.device("cuda")
    args = [torch.from_numpy(x).to(dev).requires_grad_(), torch.from_numpy(Lenv).to(dev).requires_grad_(),
            torch.from_numpy(Renv).to(dev).requires_grad_(),
            torch.from_numpy(W1[2]).requires_grad_(),                 # host operators
            torch.from_numpy(W2[2]).to(dev).requires_grad_()]         # device operators
    E = F.apply(*args)
    assert E.device.type == "cuda" and E.dtype == torch.float64
    E.backward()
    for a in args:
        assert a.grad is not None and a.grad.device == a.device and a.grad.dtype == a.dtype
    rng = np.random.default_rng(5)
    eps = 1e-4
    for i, a in enumerate(args):
        d = torch.from_numpy(rng.standard_normal(tuple(a.shape))).to(a.device)
        plus = [t.detach() + (eps * d if j == i else 0) for j, t in enumerate(args)]
        minus = [t.detach() - (eps * d if j == i else 0) for j, t in enumerate(args)]
        fd = (F.apply(*plus).item() - F.apply(*minus).item()) / (2 * eps)
        an = float((a.grad * d).sum())
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an)), (i, fd, an)
    ctx.close()


@pytest.mark.timeout(600)
def test_mpo_energy_function_gives_dE_dh_L16_chi256():
    import torch
    from paper_2505_23429_amd.api import make_mpo_energy, mpo_linear_map, open_context
    from paper_2505_23429_amd.mpo import build_mpo

    L, chi = 16, 256
    h, B = S.integrals(L, L, 1002)
    mpo = build_mpo(h, B)
    cores, labels = S.random_mps(L, L, 0, chi, 1003)
    print(f"L={L} chi={chi} R_mid={mpo.R[L // 2]}", flush=True)
    ctx = open_context(mpo, cores, labels, chi=chi)
    E0 = ctx.energy()
    F = make_mpo_energy(ctx, mpo)
    ops_of = mpo_linear_map(mpo, h)
    ht = torch.tensor(h, requires_grad=True)
    E = F.apply(ops_of(ht))
    assert abs(E.item() - E0) < 1e-10 * abs(E0)
    E.backward()
    g = ht.grad.numpy()
    assert abs(np.trace(g) - L) < 1e-9
    rng = np.random.default_rng(16)
    pairs = [(p, p) for p in range(0, L, 3)] + [tuple(rng.choice(L, 2, replace=False)) for _ in range(6)]
    for p, q in pairs:
        ref = D.one_rdm_entry(cores, int(p), int(q))
        assert abs(g[p, q] - ref) < 1e-10, (p, q, g[p, q], ref)
    # the forward follows its input: E(h + d) through the Function (new operators
    # uploaded) equals a context built from h + d, and E is linear in h
    d = rng.standard_normal((L, L)) * 1e-3
    d = 0.5 * (d + d.T)
    E1 = F.apply(ops_of(ht.detach() + torch.from_numpy(d))).item()
    assert abs((E1 - E0) - float(np.sum(d * g))) < 1e-9
    ctx.close()
    ctx2 = open_context(build_mpo(h + d, B), cores, labels, chi=chi)
    assert abs(ctx2.energy() - E1) < 1e-10 * abs(E1)
    ctx2.close()
