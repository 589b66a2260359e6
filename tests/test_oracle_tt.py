"""Pins of the tensor-train oracle: Algorithms 1 and 2 against exact
diagonalisation, invariants of the coarse problem, orthogonality, gauge."""
import numpy as np
import pytest

import seeded_inputs as S
from oracle import fock as F
from oracle import tt as T


@pytest.fixture(scope="module")
def prob6():
    h, B = S.workload_integrals(1)
    return T.Problem(h, B, 6, 0)


@pytest.fixture(scope="module")
def e_ed6():
    h, B = S.workload_integrals(1)
    return F.ed_ground(h, B, 6, 0)[0]


def _left_orth(L, N, chi, seed):
    cores, labels = S.random_mps(L, N, 0, chi, seed)
    return T.left_orthogonalize(cores, labels), labels


def test_truncation_rule():
    s = np.array([1.0, 0.5, 0.3, 0.3, 0.3, 0.1, 1e-13])
    assert T.truncation_keep(s, 10, 1e-12, 1e-10) == 6      # cutoff drops the last
    assert T.truncation_keep(s, 4, 1e-12, 1e-10) == 2       # group {0.3 x3} straddles -> dropped
    assert T.truncation_keep(s, 5, 1e-12, 1e-10) == 5       # group fits entirely
    assert T.truncation_keep(s, 2, 1e-12, 1e-10) == 2


def test_left_orthogonal_and_lq_sweep_orthonormality(prob6):
    cores, labels = _left_orth(6, 6, 16, 3001)
    for U in cores[:-1]:
        M = U.reshape(-1, U.shape[2])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() < 1e-12
    V, W = T.lq_sweep(cores, labels)
    full = T.contract_full(cores)
    for k in range(1, 6):
        M = V[k].reshape(V[k].shape[0], -1)
        assert np.abs(M @ M.T - np.eye(M.shape[0])).max() < 1e-12
    for k in range(6):
        kcopy = cores[:k] + [W[k]] + [V[j] for j in range(k + 1, 6)]
        assert np.abs(T.contract_full(kcopy) - full).max() < 1e-12


def test_retraction_is_isometry_and_heff_is_projection(prob6):
    cores, labels = _left_orth(6, 6, 16, 3002)
    V, W = T.lq_sweep(cores, labels)
    k = 2
    cur = cores[:k] + [W[k]] + [V[j] for j in range(k + 1, 6)]
    P, m = prob6.retraction(cur, k, labels[k], labels[k + 2])
    assert np.abs(P.T @ P - np.eye(P.shape[1])).max() < 1e-12
    # P x reproduces the TT with the two-site core x
    x = T.two_site(cur, k)
    y = P @ x[m]
    assert np.abs(y - prob6.to_sector(T.contract_full(cur))).max() < 1e-12
    # QN-disallowed entries of the two-site tensor vanish
    assert np.abs(x[~m]).max() == 0.0


def test_dmrg_full_rank_equals_exact_diagonalisation(prob6, e_ed6):
    cores, labels = _left_orth(6, 6, 64, 2001)
    en, cur, lab = T.dmrg2(prob6, cores, labels, 64, nsweeps=1)
    assert abs(en[-1] - e_ed6) < 1e-10


def test_dmrg_truncated_is_variational(prob6, e_ed6):
    cores, labels = _left_orth(6, 6, 16, 2002)
    en, cur, lab = T.dmrg2(prob6, cores, labels, 16, nsweeps=2)
    assert all(e >= e_ed6 - 1e-12 for e in en)
    assert max(q.shape[0] for q in lab) <= 16
    # the final TT is a proper N=6, Sz=0 state: no weight outside the sector
    full = T.contract_full(cur)
    inside = np.zeros(full.size, dtype=bool)
    inside[prob6.tidx] = True
    assert np.abs(full[~inside]).max() < 1e-12
    assert abs(prob6.energy(cur) - en[-1]) < 1e-6 * abs(en[-1]) + 1e-2


def test_a2dmrg_single_sweep_exact_at_full_rank(prob6, e_ed6):
    cores, labels = _left_orth(6, 6, 64, 2001)
    rep = T.a2dmrg_sweep(prob6, cores, labels, 64, (2, 2, 2))
    assert abs(rep.E_new - e_ed6) < 1e-10
    assert abs(rep.lam - e_ed6) < 1e-10


def test_coarse_invariants_and_exact_compression(prob6, e_ed6):
    cores, labels = _left_orth(6, 6, 16, 2003)
    En = prob6.energy(cores)
    rep = T.a2dmrg_sweep(prob6, cores, labels, 16, (2, 2, 2))
    S_, A_ = rep.S, rep.A
    assert np.allclose(np.diag(S_), 1.0, atol=1e-12)
    assert np.linalg.eigvalsh(S_).min() > -1e-12
    assert abs(A_[0, 0] - En) < 1e-10
    assert rep.lam <= min(np.diag(A_)) + 1e-12
    assert rep.lam >= e_ed6 - 1e-12 and rep.E_new >= e_ed6 - 1e-12
    assert abs(rep.c @ S_ @ rep.c - 1.0) < 1e-10
    # without truncation in Step 4 the compressed state reproduces lambda
    y = np.stack([prob6.to_sector(T.contract_full(s)) for s in rep.states], axis=1) @ rep.c
    cores2, lab2 = T.tt_svd(prob6, y, 64)
    assert abs(prob6.energy(cores2) - rep.lam) < 1e-10


def test_rank_deficient_overlap_branch():
    # duplicated update directions make the overlap singular: the eps branch
    rng = np.random.default_rng(5)
    Y = rng.standard_normal((30, 3))
    Y = np.concatenate([Y, Y[:, 1:2]], axis=1)
    H = rng.standard_normal((30, 30)); H = H + H.T
    S_, A_ = Y.T @ Y, Y.T @ H @ Y
    lam, c, rank = T.coarse_solve(S_, A_, 1e-8)
    assert rank == 3
    Q, _ = np.linalg.qr(Y[:, :3])
    ref = np.linalg.eigvalsh(Q.T @ H @ Q)[0]
    assert abs(lam - ref) < 1e-10


def test_gauge_invariance(prob6):
    cores, labels = _left_orth(6, 6, 16, 2004)
    rng = np.random.default_rng(9)
    g = [c.copy() for c in cores]
    for k in range(1, 6):
        q = labels[k]
        A = np.zeros((q.shape[0], q.shape[0]))
        for key in {tuple(r) for r in q}:
            idx = np.nonzero(np.all(q == key, axis=1))[0]
            A[np.ix_(idx, idx)] = rng.standard_normal((idx.size, idx.size)) + 3 * np.eye(idx.size)
        g[k - 1] = np.einsum("asb,bc->asc", g[k - 1], A)
        g[k] = np.einsum("bc,csd->bsd", np.linalg.inv(A), g[k])
    assert abs(prob6.energy(g) - prob6.energy(cores)) < 1e-10
    g = T.left_orthogonalize(g, labels)
    r1 = T.a2dmrg_sweep(prob6, cores, labels, 16, (3, 3))
    r2 = T.a2dmrg_sweep(prob6, g, labels, 16, (3, 3))
    assert abs(r1.E_new - r2.E_new) < 1e-9
    assert np.allclose(r1.E_local, r2.E_local, atol=1e-9)
