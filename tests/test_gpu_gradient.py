"""Backward of E = <U|H(h)|U> at L = 16, chi = 256 (the one-bond-plus-chains
gradient workload): the device's hand-written backward through the
environment chains to every MPO entry, reduced to dE/dh, against properties
that fix it at any size:
- dE/dh_pq equals the one-particle density matrix gamma_pq of the state; its
  entries are sampled from the oracle's transfer-matrix contraction;
- tr gamma = N_e and gamma is symmetric (real state);
- E is linear in h for a fixed state, so E(h + d) - E(h) = sum_pq d_pq gamma_pq
  exactly (both energies from the device forward chain)."""
import time

import numpy as np
import pytest

import seeded_inputs as S
from oracle import density as D

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_gradient_L16_chi256():
    from paper_2505_23429_amd.api import open_context
    from paper_2505_23429_amd.mpo import build_mpo, h_gradient

    L, chi = 16, 256
    h, B = S.integrals(L, L, 1002)
    mpo = build_mpo(h, B)
    cores, labels = S.random_mps(L, L, 0, chi, 1003)
    print(f"L={L} chi={chi} R_mid={mpo.R[L // 2]}", flush=True)
    ctx = open_context(mpo, cores, labels, chi=chi)
    t = time.perf_counter()
    E0 = ctx.energy()
    t_fwd = time.perf_counter() - t
    t = time.perf_counter()
    E, gops = ctx.mpo_gradient(mpo)
    t_bwd = time.perf_counter() - t
    print(f"forward (energy chain) {t_fwd:.3f}s, forward+backward {t_bwd:.3f}s", flush=True)
    g = h_gradient(mpo, gops)
    assert abs(E - E0) < 1e-10 * abs(E0)
    assert abs(np.trace(g) - L) < 1e-9
    assert np.abs(g - g.T).max() < 1e-10
    # sampled entries against the oracle (all diagonal entries, seeded off-diagonal pairs)
    rng = np.random.default_rng(16)
    pairs = [(p, p) for p in range(L)] + [tuple(rng.choice(L, 2, replace=False)) for _ in range(12)]
    for p, q in pairs:
        ref = D.one_rdm_entry(cores, int(p), int(q))
        assert abs(g[p, q] - ref) < 1e-10, (p, q, g[p, q], ref)
    ctx.close()
    # linearity in h (fixed state)
    d = rng.standard_normal((L, L)) * 1e-3
    d = 0.5 * (d + d.T)
    ctx2 = open_context(build_mpo(h + d, B), cores, labels, chi=chi)
    E1 = ctx2.energy()
    ctx2.close()
    assert abs((E1 - E0) - float(np.sum(d * g))) < 1e-9
