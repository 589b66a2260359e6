"""Pins of the oracle's additive two-level method for the linear-system functional
J(X) = 1/2 <X,AX> - <F,X> (eq. energy_lin), A symmetric positive definite.

Checked against: the exact solution of A X = F (J* = -1/2 <F, A^{-1} F>, reached in
one global iteration at full TT rank), the optimality conditions of the coarse
problem (its gradient vanishes on the span of the updates; its minimum is below the
best multiple of every update and below the iterate), and the identity between a
micro-step's minimum and J of the update it produces (the retraction is an
isometry, so J(P w) = 1/2 w.P^T A P w - w.P^T F).
"""
import numpy as np
import pytest

import seeded_inputs as S
from oracle import tt as T


def _problem(L, seed, chi, mps_seed, chi_f):
    hs, B, sigma, F, Fl = S.linear_system(L, L, seed, chi_f)
    prob = T.Problem(hs, B, L, 0)
    cores, labels = S.random_mps(L, L, 0, chi, mps_seed)
    cores = S.unit_tt(cores)
    oc = T.left_orthogonalize(cores, labels)
    return prob, oc, labels, F, Fl, sigma


def test_shifted_operator_is_positive_definite():
    """The input recipe's shift makes A >= 1 on the sector (here well above it)."""
    for L, seed in ((4, 41), (6, 1001)):
        hs, B, sigma, _, _ = S.linear_system(L, L, seed, 4)
        w = np.linalg.eigvalsh(T.Problem(hs, B, L, 0).H)
        assert w[0] >= 1.0
        h, _ = S.integrals(L, L, seed)
        w0 = np.linalg.eigvalsh(T.Problem(h, B, L, 0).H)
        assert np.allclose(w, w0 + sigma, atol=1e-9)  # a pure shift on the sector


@pytest.mark.parametrize("sites", [2, 1])
def test_linear_full_rank_single_sweep_exact(sites):
    """At full rank the middle subdomain's local space is the whole sector (two-site:
    already the first subdomain's second window, sites 1-2): one global iteration
    reaches the exact minimum J* = -1/2 F.A^{-1}F."""
    L = 6
    prob, oc, labels, F, Fl, _ = _problem(L, 1001, 64, 1002, 8)
    f = prob.to_sector(T.contract_full(F))
    j_star = -0.5 * f @ np.linalg.solve(prob.H, f)
    r = T.a2dmrg_lin_sweep(prob, oc, labels, 64, (2, 2, 2), F, sites=sites)
    assert abs(r.E_local[1] - j_star) < 1e-10 * abs(j_star)
    if sites == 1:
        # site 1's space (4 x 4 x 16 of the 1024 right states) is not the whole sector
        assert r.E_local[0] > j_star + 1e-6 * abs(j_star)
    assert abs(r.J_coarse - j_star) < 1e-10 * abs(j_star)
    assert abs(r.J_new - j_star) < 1e-10 * abs(j_star)


@pytest.mark.parametrize("L,seed,chi,lengths,mps_seed,sites",
                         [(6, 1001, 16, (2, 2, 2), 19, 2), (8, 1008, 24, (2, 3, 3), 27, 2),
                          (6, 1006, 12, (1, 2, 3), 21, 1), (8, 1008, 24, (3, 1, 4), 27, 1)])
def test_linear_sweep_invariants(L, seed, chi, lengths, mps_seed, sites):
    prob, oc, labels, F, Fl, _ = _problem(L, seed, chi, mps_seed, 6)
    f = prob.to_sector(T.contract_full(F))
    # without truncation (room for every rank) each update is exactly P w
    r = T.a2dmrg_lin_sweep(prob, oc, labels, 8 * chi, lengths, F, sites=sites)
    Y = np.stack([prob.to_sector(T.contract_full(st)) for st in r.states], axis=1)
    for j in range(1, Y.shape[1]):
        y = Y[:, j]
        assert abs(0.5 * y @ prob.H @ y - f @ y - r.E_local[j - 1]) < 1e-9 * abs(r.E_local[j - 1])
        # the coarse minimum is below the best multiple of every update
        assert r.J_coarse <= -0.5 * (f @ y) ** 2 / (y @ prob.H @ y) + 1e-10
    assert r.J_coarse <= r.J_before + 1e-10
    # stationarity on the span: the coarse gradient A c - b vanishes in every kept direction
    w, V = np.linalg.eigh(r.S)
    keep = w >= 1e-8 * w.max()
    g = V[:, keep].T @ (r.A @ r.c - r.b)
    assert np.abs(g).max() < 1e-9 * max(1.0, np.abs(r.b).max())
    # with room for the combination's ranks the compression is exact
    assert abs(r.J_new - r.J_coarse) < 1e-9 * abs(r.J_coarse)
    # with truncation to the iterate's chi, the result is still a TT of rank <= chi
    rt = T.a2dmrg_lin_sweep(prob, oc, labels, chi, lengths, F, sites=sites)
    assert max(c.shape[2] for c in rt.cores) <= chi
    assert rt.J_coarse <= rt.J_before + 1e-10


@pytest.mark.parametrize("L,seed,chi,lengths,mps_seed,sites",
                         [(6, 1001, 16, (2, 2, 2), 19, 2), (8, 1008, 24, (2, 3, 3), 27, 2),
                          (6, 1006, 12, (1, 2, 3), 21, 1), (8, 1008, 24, (3, 1, 4), 27, 1)])
def test_linear_chain_equals_dense_oracle(L, seed, chi, lengths, mps_seed, sites):
    """The environment-chain version (conjugate gradients on the chain product, P^T F
    from overlap environments, TT sandwiches, TT rounding) reports what the dense one
    does."""
    from oracle import chain as CH
    from oracle import mpo as OM

    prob, oc, labels, F, Fl, _ = _problem(L, seed, chi, mps_seed, 6)
    hs, B, _, _, _ = S.linear_system(L, L, seed, 6)
    rd = T.a2dmrg_lin_sweep(prob, oc, labels, chi, lengths, F, sites=sites)
    rc = CH.a2dmrg_lin_sweep(OM.build_mpo(hs, B), oc, labels, chi, lengths, F, sites=sites, tol=1e-13)
    sc = abs(rd.J_before) + abs(rd.J_new)
    assert abs(rd.J_before - rc.J_before) < 1e-10 * sc
    assert np.abs(np.array(rd.E_local) - np.array(rc.E_local)).max() < 1e-9 * sc
    assert np.abs(rd.S - rc.S).max() < 1e-10
    assert np.abs(rd.A - rc.A).max() < 1e-9 * np.abs(rd.A).max()
    assert np.abs(rd.b - rc.b).max() < 1e-9 * np.abs(rd.b).max()
    dc = rd.c - rc.c
    assert np.sqrt(abs(dc @ rd.S @ dc)) < 1e-8 * np.sqrt(rd.c @ rd.S @ rd.c)
    assert rd.rankS == rc.rankS
    assert abs(rd.J_coarse - rc.J_coarse) < 1e-9 * sc and abs(rd.J_new - rc.J_new) < 1e-9 * sc
    assert [q.shape[0] for q in rd.labels] == [q.shape[0] for q in rc.labels]
