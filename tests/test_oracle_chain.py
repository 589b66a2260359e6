"""Pins of the environment-chain oracle (oracle.mpo, oracle.chain) and of the
oracle's Lanczos solver and truncated block SVD.

Each check is against something fixed independently of the code under test:
the Fock-space Hamiltonian built from the Jordan-Wigner definition, exact
diagonalisation, the dense-vector oracle (explicit P^T H P and dense coarse
matrices), the Eckart-Young theorem, the full SVD of the unblocked matrix,
and dense eigensolvers.
"""
import numpy as np
import pytest

import seeded_inputs as S
from oracle import chain as CH
from oracle import fock as F
from oracle import mpo as OM
from oracle import tt as T
from oracle.lanczos import lanczos_lowest


def _gauge(S_, A_, c):
    d = np.sign(S_[0])
    d[0] = 1.0
    d[d == 0] = 1.0
    Sg, Ag, cg = S_ * np.outer(d, d), A_ * np.outer(d, d), c * d
    i = int(np.argmax(np.abs(cg)))
    return Sg, Ag, (-cg if cg[i] < 0 else cg)


# ---------------------------------------------------------------------------
# oracle MPO
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("L", [2, 3])
def test_mpo_equals_term_by_term_hamiltonian(L):
    h, B = S.integrals(L, L, 500 + L)
    W = OM.mpo_to_matrix(OM.build_mpo(h, B))
    eri = np.einsum("kpq,krs->pqrs", B, B)
    assert np.abs(W - F.hamiltonian_direct(h, eri)).max() < 1e-12


@pytest.mark.parametrize("L", [4, 5])
def test_mpo_equals_fock_hamiltonian(L):
    h, B = S.integrals(L, L, 600 + L)
    W = OM.mpo_to_matrix(OM.build_mpo(h, B))
    Hf = F.hamiltonian(h, B, F.all_states(L), dense=True)
    assert np.abs(W - Hf).max() < 1e-11


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6, 7, 8])
def test_mpo_bond_dimension(L):
    """Identity and done channels, 4L single operators, and 8m^2 - 2m pairs on the
    smaller side: no redundant channel."""
    h, B = S.integrals(L, L, 700 + L)
    m = OM.build_mpo(h, B)
    want = [1] + [2 + 4 * L + 8 * min(l, L - l) ** 2 - 2 * min(l, L - l) for l in range(1, L)] + [1]
    assert m.R == want


def test_mpo_energy_of_random_state_L8():
    """<psi|H|psi> through the chain of the oracle MPO equals the sector matrix at
    L = 8 (beyond the full-matrix checks: pair channels on both sides of the switch)."""
    L = 8
    h, B = S.integrals(L, L, 1008)
    mpo = OM.build_mpo(h, B)
    ops = [CH.site_ops(mpo, k) for k in range(L)]
    cores, labels = S.random_mps(L, L, 0, 20, 31)
    prob = T.Problem(h, B, L, 0)
    assert abs(CH.chain_energy(mpo, ops, cores) - prob.energy(cores)) < 1e-10


# ---------------------------------------------------------------------------
# contractions
# ---------------------------------------------------------------------------

def test_chain_product_is_projected_hamiltonian():
    """H_eff x from environments equals P^T H P x with the explicit retraction."""
    L, k = 6, 2
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
    for i in range(L - 1, k + 1, -1):
        Re = CH.env_right(Re, cur[i], ops[i], cur[i])
    P, m = prob.retraction(cur, k, labels[k], labels[k + 2])
    x = np.zeros(m.shape)
    x[m] = np.random.default_rng(5).standard_normal(int(m.sum()))
    y = CH.heff_apply(Le, ops[k], ops[k + 1], Re, x)
    assert np.abs(y[m] - P.T @ (prob.H @ (P @ x[m]))).max() < 1e-10
    assert np.abs(y[~m]).max() < 1e-12


def test_chain_sandwich_is_dense_inner_product():
    L = 6
    h, B = S.workload_integrals(1)
    mpo = OM.build_mpo(h, B)
    ops = [CH.site_ops(mpo, i) for i in range(L)]
    prob = T.Problem(h, B, L, 0)
    a, _ = S.random_mps(L, L, 0, 12, 41)
    b, _ = S.random_mps(L, L, 0, 9, 42)
    ya, yb = prob.to_sector(T.contract_full(a)), prob.to_sector(T.contract_full(b))
    E, N = CH.chain_sandwich(ops, a, b)
    assert abs(N - ya @ yb) < 1e-10 * max(1.0, abs(N))
    assert abs(E - ya @ prob.H @ yb) < 1e-10 * max(1.0, abs(E))


# ---------------------------------------------------------------------------
# Lanczos, truncated block SVD, TT rounding
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,seed", [(60, 1), (200, 2), (400, 3)])
def test_lanczos_lowest_matches_dense_eigensolver(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.sort(rng.uniform(-5.0, 5.0, n))
    ev[1] = ev[0] + 0.05  # small gap above the ground state
    H = (Q * ev) @ Q.T
    theta, u = lanczos_lowest(lambda v: H @ v, rng.standard_normal(n), tol=1e-11, maxiter=n)
    assert abs(theta - ev[0]) < 1e-10
    assert abs(abs(u @ Q[:, 0]) - 1.0) < 1e-10
    assert np.linalg.norm(H @ u - theta * u) <= 1e-10


def test_lanczos_exhausts_small_krylov_space():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((9, 9))
    H = A + A.T
    theta, u = lanczos_lowest(lambda v: H @ v, rng.standard_normal(9), tol=1e-14, maxiter=500)
    assert abs(theta - np.linalg.eigvalsh(H)[0]) < 1e-12


def _block_matrix(seed):
    rng = np.random.default_rng(seed)
    rq = rng.integers(0, 3, size=(40, 2))
    cq = rng.integers(0, 3, size=(35, 2))
    M = rng.standard_normal((40, 35)) * np.all(rq[:, None, :] == cq[None, :, :], axis=-1)
    return M, rq, cq


@pytest.mark.parametrize("chi", [3, 7, 12])
def test_truncated_block_svd_is_best_approximation(chi):
    """Eckart-Young: the kept singular values are the chi largest of the whole
    matrix, and the discarded weight equals ||M - U S V^T||_F^2."""
    M, rq, cq = _block_matrix(11 + chi)
    U, s, Vt, qn, disc = T.sector_svd(M, rq, cq, chi, cutoff=1e-12, tau=1e-10)
    full = np.linalg.svd(M, compute_uv=False)
    full = full[full > 1e-12 * full[0]]
    assert s.size == min(chi, full.size)
    assert np.allclose(np.sort(s)[::-1], full[:s.size], rtol=0, atol=1e-12)
    assert abs(disc - np.sum(full[s.size:] ** 2)) < 1e-10
    assert abs(np.linalg.norm(M - (U * s) @ Vt) ** 2 - disc) < 1e-10
    assert np.abs(U.T @ U - np.eye(s.size)).max() < 1e-12
    assert np.abs(Vt @ Vt.T - np.eye(s.size)).max() < 1e-12
    # every kept vector lives in one charge block, the one of its label
    for j in range(s.size):
        assert np.all(np.all(rq[np.abs(U[:, j]) > 0] == qn[j], axis=1))
        assert np.all(np.all(cq[np.abs(Vt[j]) > 0] == qn[j], axis=1))


def test_tt_rounding_of_direct_sum():
    """Without truncation the rounded direct sum is the linear combination of the
    dense vectors; with truncation it equals the TT-SVD of that vector."""
    L = 6
    h, B = S.workload_integrals(1)
    prob = T.Problem(h, B, L, 0)
    sts, labs = [], []
    for seed in (1, 2, 3):
        c_, l_ = S.random_mps(L, L, 0, 6, seed)
        sts.append(c_)
        labs.append(l_)
    coef = np.array([0.7, -1.3, 0.4])
    dense = sum(c * prob.to_sector(T.contract_full(st)) for c, st in zip(coef, sts))
    sc, sl = CH.tt_direct_sum(sts, coef, labs)
    assert np.abs(prob.to_sector(T.contract_full(sc)) - dense).max() < 1e-12
    rc, rl = CH.tt_round(sc, sl, 64)
    assert np.abs(prob.to_sector(T.contract_full(rc)) - dense).max() < 1e-11
    tc, tl = CH.tt_round(sc, sl, 8)
    ref, _ = T.tt_svd(prob, dense, 8)
    assert [q.shape[0] for q in tl] == [c.shape[0] for c in ref] + [1]
    assert abs(prob.energy(tc) - prob.energy(ref)) < 1e-10


# ---------------------------------------------------------------------------
# whole algorithms
# ---------------------------------------------------------------------------

def test_chain_dmrg_full_rank_equals_ed():
    """Algorithm 1 through environments and the Lanczos solver reaches the exact
    ground state at full rank."""
    h, B = S.workload_integrals(1)
    mpo = OM.build_mpo(h, B)
    cores, labels = S.random_mps(6, 6, 0, 64, 2001)
    cores = T.left_orthogonalize(cores, labels)
    en, _, _ = CH.dmrg2(mpo, cores, labels, 64, nsweeps=1)
    assert abs(en[-1] - F.ed_ground(h, B, 6, 0)[0]) < 1e-10


def test_chain_dmrg_truncated_equals_dense_oracle():
    h, B = S.workload_integrals(1)
    mpo = OM.build_mpo(h, B)
    prob = T.Problem(h, B, 6, 0)
    cores, labels = S.random_mps(6, 6, 0, 16, 2002)
    cores = T.left_orthogonalize(cores, labels)
    e1, _, _ = CH.dmrg2(mpo, cores, labels, 16, nsweeps=2)
    e2, _, _ = T.dmrg2(prob, cores, labels, 16, nsweeps=2)
    assert np.abs(np.array(e1) - np.array(e2)).max() < 1e-9


@pytest.mark.parametrize("L,seed,chi,lengths,mps_seed", [(6, 1001, 16, (2, 2, 2), 19), (8, 1008, 16, (3, 3, 2), 19),
                                                          (8, 1008, 24, (2, 3, 3), 27)])
def test_chain_a2dmrg_equals_dense_oracle(L, seed, chi, lengths, mps_seed):
    """One global iteration of Algorithm 2 through environment chains equals the
    dense-vector oracle (explicit P^T H P local problems, dense coarse matrices,
    TT-SVD of the dense combination)."""
    h, B = S.integrals(L, L, seed)
    mpo = OM.build_mpo(h, B)
    prob = T.Problem(h, B, L, 0)
    cores, labels = S.random_mps(L, L, 0, chi, mps_seed)
    oc = T.left_orthogonalize(cores, labels)
    rd = T.a2dmrg_sweep(prob, oc, labels, chi, lengths)
    rc = CH.a2dmrg_sweep(mpo, oc, labels, chi, lengths)
    assert abs(rc.E_before - prob.energy(oc)) < 1e-11
    assert np.abs(np.array(rd.E_local) - np.array(rc.E_local)).max() < 1e-10
    Sd, Ad, cd = _gauge(rd.S, rd.A, rd.c)
    Sc, Ac, cc = _gauge(rc.S, rc.A, rc.c)
    assert np.abs(Sd - Sc).max() < 1e-10
    assert np.abs(Ad - Ac).max() < 1e-9
    assert np.abs(cd - cc).max() < 1e-9
    assert rd.rankS == rc.rankS
    assert abs(rd.lam - rc.lam) < 1e-10
    assert abs(rd.E_new - rc.E_new) < 1e-10
    assert abs(prob.energy(rc.cores) - rd.E_new) < 1e-10
    assert max(q.shape[0] for q in rc.labels) <= chi


def test_chain_a2dmrg_full_rank_single_sweep_exact():
    """At full rank one global iteration reaches the exact ground state."""
    h, B = S.workload_integrals(1)
    mpo = OM.build_mpo(h, B)
    cores, labels = S.random_mps(6, 6, 0, 64, 2001)
    oc = T.left_orthogonalize(cores, labels)
    rc = CH.a2dmrg_sweep(mpo, oc, labels, 64, (2, 2, 2))
    assert abs(rc.E_new - F.ed_ground(h, B, 6, 0)[0]) < 1e-10


# ---------------------------------------------------------------------------
# Extension One (the K lowest eigenvectors of every subdomain's last micro-step)
# ---------------------------------------------------------------------------

def test_several_lowest_eigenpairs_match_dense_solver():
    """The chain oracle's several-root solver (ARPACK above 400 unknowns) against eigh."""
    from oracle import chain as CHm

    L, k = 8, 3
    h, B = S.integrals(L, L, 1008)
    mpo = OM.build_mpo(h, B)
    ops = [CHm.site_ops(mpo, i) for i in range(L)]
    prob = T.Problem(h, B, L, 0)
    cores, labels = S.random_mps(L, L, 0, 24, 27)
    cores = T.left_orthogonalize(cores, labels)
    V, W = T.lq_sweep(cores, labels)
    cur = cores[:k] + [W[k]] + [V[j] for j in range(k + 1, L)]
    Le = np.ones((1, 1, 1))
    for i in range(k):
        Le = CHm.env_left(Le, cur[i], ops[i], cur[i])
    Re = np.ones((1, 1, 1))
    for i in range(L - 1, k + 1, -1):
        Re = CHm.env_right(Re, cur[i], ops[i], cur[i])
    x0 = np.einsum("asb,btc->astc", cur[k], cur[k + 1])
    pairs, _ = CHm.local_solve_k(Le, ops[k], ops[k + 1], Re, x0, labels[k], labels[k + 2], 3)
    ref = prob.local_solve_k(cur, k, labels[k], labels[k + 2], 3)
    assert int(T.x_mask(labels[k], labels[k + 2]).sum()) > 400  # the ARPACK branch
    for (t1, x1), (t2, x2) in zip(pairs, ref):
        assert abs(t1 - t2) < 1e-10
        assert abs(abs(np.sum(x1 * x2)) - 1.0) < 1e-8


@pytest.mark.parametrize("L,seed,chi,lengths,mps_seed", [(6, 1001, 16, (2, 2, 2), 19), (8, 1008, 24, (2, 3, 3), 27)])
def test_extension_one_chain_equals_dense_and_lowers_the_coarse_energy(L, seed, chi, lengths, mps_seed):
    """Two kept eigenvectors per subdomain: the environment-chain and dense-vector
    oracles agree, the coarse space holds 2P + 1 states, and enriching it can only
    lower the coarse eigenvalue (the plain method's states are among them)."""
    h, B = S.integrals(L, L, seed)
    mpo = OM.build_mpo(h, B)
    prob = T.Problem(h, B, L, 0)
    cores, labels = S.random_mps(L, L, 0, chi, mps_seed)
    oc = T.left_orthogonalize(cores, labels)
    rd = T.a2dmrg_sweep(prob, oc, labels, chi, lengths, n_eig=2)
    rc = CH.a2dmrg_sweep(mpo, oc, labels, chi, lengths, n_eig=2)
    r1 = T.a2dmrg_sweep(prob, oc, labels, chi, lengths)
    assert rd.S.shape == (2 * len(lengths) + 1,) * 2
    Sd, Ad, cd = _gauge(rd.S, rd.A, rd.c)
    Sc, Ac, cc = _gauge(rc.S, rc.A, rc.c)
    assert np.abs(Sd - Sc).max() < 1e-10 and np.abs(Ad - Ac).max() < 1e-9 and np.abs(cd - cc).max() < 1e-9
    assert abs(rd.lam - rc.lam) < 1e-10 and abs(rd.E_new - rc.E_new) < 1e-10
    assert np.abs(np.array(rd.E_local) - np.array(r1.E_local)).max() < 1e-10
    assert rd.lam <= r1.lam + 1e-12
    # the plain method's coarse states are the enriched space's states 0, 1, 3, 5, ...
    sel = [0] + [1 + 2 * j for j in range(len(lengths))]
    assert np.abs(np.abs(rd.S[np.ix_(sel, sel)]) - np.abs(r1.S)).max() < 1e-10
