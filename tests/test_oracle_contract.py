"""Pins of the einsum contractions: environments and matvec against the
explicit projection P^T M P of an independently contracted operator."""
import numpy as np

import seeded_inputs as S
from oracle import contract as C
from oracle import tt as T


def _random_mpo(L, R, seed):
    rng = np.random.default_rng(seed)
    dims = [1] + [R] * (L - 1) + [1]
    return [rng.standard_normal((dims[k], 4, 4, dims[k + 1])) for k in range(L)]


def _mpo_matrix(W):
    """Plain contraction of an MPO to its 4^L matrix (test-side, no environments)."""
    M = W[0][0]
    for Wk in W[1:]:
        D = M.shape[0]
        M = np.einsum("xyA,AusB->xuysB", M, Wk).reshape(D * 4, D * 4, -1)
    return M[:, :, 0]


def test_env_chain_and_matvec_equal_projected_operator():
    L = 5
    W = _random_mpo(L, 3, 1)
    Mfull = _mpo_matrix(W)
    cores, labels = S.random_mps(L, 4, 0, 8, 17)
    cores = T.left_orthogonalize(cores, labels)
    V, Wc = T.lq_sweep(cores, labels)
    k = 1
    cur = cores[:k] + [Wc[k]] + [V[j] for j in range(k + 1, L)]
    Lenv = np.ones((1, 1, 1))
    for j in range(k):
        Lenv = C.env_left(Lenv, cur[j], W[j], cur[j])
    Renv = np.ones((1, 1, 1))
    for j in range(L - 1, k + 1, -1):
        Renv = C.env_right(Renv, cur[j], W[j], cur[j])
    Heff = C.heff_matrix(Lenv, W[k], W[k + 1], Renv)
    # explicit retraction on the full space (no sector restriction)
    PhiL = T.left_block(cur, k)
    PhiR = T.right_block(cur, k + 2)
    P = np.kron(PhiL, np.kron(np.eye(16), PhiR.T))
    ref = P.T @ Mfull @ P
    assert np.abs(Heff - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())
    x = np.random.default_rng(2).standard_normal((cur[k].shape[0], 4, 4, cur[k + 1].shape[2]))
    y = C.heff_apply(Lenv, W[k], W[k + 1], Renv, x)
    assert np.abs(y.reshape(-1) - Heff @ x.reshape(-1)).max() < 1e-10 * max(1.0, np.abs(y).max())


def test_overlap_chain_is_inner_product():
    L = 5
    a, la = S.random_mps(L, 4, 0, 8, 21)
    b, lb = S.random_mps(L, 4, 0, 6, 22)
    E = np.ones((1, 1))
    for j in range(L):
        E = C.overlap_left(E, a[j], b[j])
    ref = T.contract_full(a) @ T.contract_full(b)
    assert abs(E[0, 0] - ref) < 1e-10 * max(1.0, abs(ref))
    E = np.ones((1, 1))
    for j in range(L - 1, -1, -1):
        E = C.overlap_right(E, a[j], b[j])
    assert abs(E[0, 0] - ref) < 1e-10 * max(1.0, abs(ref))


def test_gradients_by_directional_finite_differences():
    rng = np.random.default_rng(3)
    rl, rr, Rl, Rm, Rr = 3, 4, 2, 3, 2
    Lenv = rng.standard_normal((rl, Rl, rl))
    Renv = rng.standard_normal((rr, Rr, rr))
    W1 = rng.standard_normal((Rl, 4, 4, Rm))
    W2 = rng.standard_normal((Rm, 4, 4, Rr))
    x = rng.standard_normal((rl, 4, 4, rr))
    E, gx, gL, gW1, gW2, gR = C.heff_grads(Lenv, W1, W2, Renv, x)

    def En(Lv=Lenv, w1=W1, w2=W2, Rv=Renv, xv=x):
        return float(np.sum(xv * C.heff_apply(Lv, w1, w2, Rv, xv)))

    d = 1e-6
    for g, name in [(gx, "x"), (gL, "L"), (gW1, "W1"), (gW2, "W2"), (gR, "R")]:
        dirn = rng.standard_normal(g.shape)
        kw = {"x": "xv", "L": "Lv", "W1": "w1", "W2": "w2", "R": "Rv"}[name]
        base = {"xv": x, "Lv": Lenv, "w1": W1, "w2": W2, "Rv": Renv}[kw]
        fd = (En(**{kw: base + d * dirn}) - En(**{kw: base - d * dirn})) / (2 * d)
        assert abs(fd - np.sum(g * dirn)) < 1e-6 * max(1.0, abs(fd)), name


def test_sampled_rows_match_full_matvec():
    Lenv, W1s, W2s, Renv, x = S.heff_operands(6, 5, 4, 7, 3, seed=4)
    W1 = C.dense_core(*W1s, 4, 7)
    W2 = C.dense_core(*W2s, 7, 3)
    # product layouts: L[A][a'][a], R[C][b'][b]  ->  oracle layout [a',A,a]
    y = C.heff_apply(Lenv.transpose(1, 0, 2), W1, W2, Renv.transpose(1, 0, 2), x)
    rows = [Lenv[:, i, :] for i in (0, 3)]
    cols = [Renv[:, j, :] for j in (1, 4)]
    ys = C.heff_rows(rows, x, W1s, W2s, 7, 3, cols)
    for ii, i in enumerate((0, 3)):
        for jj, j in enumerate((1, 4)):
            assert np.abs(ys[ii, jj] - y[i, :, :, j]).max() < 1e-12
