"""Pins of the oracle's one-site additive two-level DMRG (Algorithm 2, one-site branch).

Checked against what is fixed independently of the code under test: the
explicit one-site retraction P^T H P, the QR factorisation's defining
properties, exact diagonalisation, the variational principle (every one-site
update lies exactly in the coarse space, so the coarse eigenvalue cannot exceed
its energy), and the dense-vector oracle for the environment-chain one.
"""
import numpy as np
import pytest

import seeded_inputs as S
from oracle import chain as CH
from oracle import fock as F
from oracle import mpo as OM
from oracle import tt as T


def _gauge(S_, A_, c):
    d = np.sign(S_[0])
    d[0] = 1.0
    d[d == 0] = 1.0
    Sg, Ag, cg = S_ * np.outer(d, d), A_ * np.outer(d, d), c * d
    i = int(np.argmax(np.abs(cg)))
    return Sg, Ag, (-cg if cg[i] < 0 else cg)


@pytest.mark.parametrize("k", [0, 2, 5])
def test_one_site_chain_product_is_projected_hamiltonian(k):
    """The one-site operator from environments equals P^T H P with the explicit
    one-site retraction, at the first, an interior and the last site."""
    L = 6
    h, B = S.workload_integrals(1)
    mpo = OM.build_mpo(h, B)
    ops = [CH.site_ops(mpo, i) for i in range(L)]
    prob = T.Problem(h, B, L, 0)
    cores, labels = S.random_mps(L, L, 0, 16, 3002)
    cores = T.left_orthogonalize(cores, labels)
    V, W = T.lq_sweep(cores, labels)
    cur = cores[:k] + [W[k]] + [V[j] for j in range(k + 1, L)]
    Le = np.ones((1, 1, 1))
    for i in range(k):
        Le = CH.env_left(Le, cur[i], ops[i], cur[i])
    Re = np.ones((1, 1, 1))
    for i in range(L - 1, k, -1):
        Re = CH.env_right(Re, cur[i], ops[i], cur[i])
    P, m = prob.retraction1(cur, k, labels[k], labels[k + 1])
    # the retraction of a k-orthogonal TT is an isometry on the allowed entries
    assert np.abs(P.T @ P - np.eye(P.shape[1])).max() < 1e-12
    x = np.zeros(m.shape)
    x[m] = np.random.default_rng(9 + k).standard_normal(int(m.sum()))
    y = CH.heff1_apply(Le, ops[k], Re, x)
    assert np.abs(y[m] - P.T @ (prob.H @ (P @ x[m]))).max() < 1e-10
    assert np.abs(y[~m]).max() < 1e-12


def test_qr_move_is_a_charge_block_qr():
    """Q R = x, Q left-orthogonal, R upper triangular within each charge block, and Q
    only has entries that the bond charges allow."""
    L = 6
    cores, labels = S.random_mps(L, L, 0, 16, 77)
    for k in range(L - 1):
        x = cores[k]
        Q, R = T.qr_left_core(x, labels[k], labels[k + 1])
        r, n, r2 = x.shape
        assert np.abs(np.einsum("asb,bc->asc", Q, R) - x).max() < 1e-12
        Qm = Q.reshape(r * n, r2)
        assert np.abs(Qm.T @ Qm - np.eye(r2)).max() < 1e-12
        assert np.abs(Q[~T.x1_mask(labels[k], labels[k + 1])]).max(initial=0.0) == 0.0
        for q in {tuple(v) for v in labels[k + 1]}:
            cols = np.nonzero(np.all(labels[k + 1] == q, axis=1))[0]
            assert np.abs(np.tril(R[np.ix_(cols, cols)], -1)).max(initial=0.0) < 1e-14


@pytest.mark.parametrize("L,seed,chi,lengths,mps_seed",
                         [(6, 1001, 16, (2, 2, 2), 19), (6, 1006, 12, (1, 2, 3), 21), (8, 1008, 24, (2, 3, 3), 27)])
def test_one_site_sweep_invariants(L, seed, chi, lengths, mps_seed):
    """Every one-site update has the bond dimensions of the iterate and the energy of
    its last micro-step (the retraction is an isometry); it lies in the coarse space,
    so lambda is at most every update's energy and the iterate's; with room for the
    rank of the combination the compression is exact (E_after = lambda)."""
    h, B = S.integrals(L, L, seed)
    prob = T.Problem(h, B, L, 0)
    cores, labels = S.random_mps(L, L, 0, chi, mps_seed)
    oc = T.left_orthogonalize(cores, labels)
    E0 = prob.energy(oc)
    r = T.a2dmrg_sweep(prob, oc, labels, 4 * chi, lengths, sites=1)
    assert len(r.states) == len(lengths) + 1
    for j, st in enumerate(r.states[1:]):
        assert [c.shape for c in st] == [c.shape for c in oc]
        assert abs(prob.energy(st) - r.E_local[j]) < 1e-10
    assert r.lam <= min(E0, min(r.E_local)) + 1e-12
    assert abs(r.E_new - r.lam) < 1e-10
    # Extension One: the enriched space holds the plain one, so lambda can only drop
    r2 = T.a2dmrg_sweep(prob, oc, labels, 4 * chi, lengths, sites=1, n_eig=2)
    assert len(r2.states) == 2 * len(lengths) + 1
    assert r2.lam <= r.lam + 1e-12


def test_one_site_full_rank_single_sweep_exact():
    """At full TT rank the bonds on both sides of a middle site (site 2 or 3 at L = 6)
    carry every state of their side that the sector can complete, so that site's
    one-site space is the whole sector: the middle subdomain's Ritz value, lambda and
    the compressed iterate are the ED ground energy after one global iteration, while
    the first subdomain (site 0: a 16-dimensional space) stays above it."""
    L = 6
    h, B = S.workload_integrals(1)
    e_ed = F.ed_ground(h, B, L, 0)[0]
    prob = T.Problem(h, B, L, 0)
    cores, labels = S.random_mps(L, L, 0, 64, 1002)
    oc = T.left_orthogonalize(cores, labels)
    r = T.a2dmrg_sweep(prob, oc, labels, 64, (2, 2, 2), sites=1)
    assert abs(r.E_local[1] - e_ed) < 1e-10
    assert r.E_local[0] > e_ed + 1e-3
    assert abs(r.lam - e_ed) < 1e-10
    assert abs(r.E_new - e_ed) < 1e-10


@pytest.mark.parametrize("L,seed,chi,lengths,mps_seed,n_eig",
                         [(6, 1001, 16, (2, 2, 2), 19, 1), (6, 1006, 12, (1, 2, 3), 21, 1),
                          (8, 1008, 24, (2, 3, 3), 27, 1), (8, 1008, 16, (3, 3, 2), 19, 2)])
def test_one_site_chain_equals_dense_oracle(L, seed, chi, lengths, mps_seed, n_eig):
    """The environment-chain one-site sweep (Lanczos, TT sandwiches, TT rounding of
    the direct sum) reports what the dense-vector one does."""
    h, B = S.integrals(L, L, seed)
    mpo = OM.build_mpo(h, B)
    prob = T.Problem(h, B, L, 0)
    cores, labels = S.random_mps(L, L, 0, chi, mps_seed)
    oc = T.left_orthogonalize(cores, labels)
    rd = T.a2dmrg_sweep(prob, oc, labels, chi, lengths, sites=1, n_eig=n_eig)
    rc = CH.a2dmrg_sweep(mpo, oc, labels, chi, lengths, sites=1, n_eig=n_eig, tol=1e-12)
    assert np.abs(np.array(rd.E_local) - np.array(rc.E_local)).max() < 1e-10
    Sd, Ad, cd = _gauge(rd.S, rd.A, rd.c)
    Sc, Ac, cc = _gauge(rc.S, rc.A, rc.c)
    assert np.abs(Sd - Sc).max() < 1e-9 and np.abs(Ad - Ac).max() < 1e-8 and np.abs(cd - cc).max() < 1e-8
    assert rd.rankS == rc.rankS
    assert abs(rd.lam - rc.lam) < 1e-10 and abs(rd.E_new - rc.E_new) < 1e-10
    assert [q.shape[0] for q in rd.labels] == [q.shape[0] for q in rc.labels]
