"""Einsum definitions of the contractions on the hot path (Appendix A).

Index conventions follow the environment definitions eq. env_L / eq. env_R:
an environment is ``E[k, K, k']`` = (bra bond, operator bond, ket bond); an MPO
core (eq. MPO) is ``W[K, s_out, s_in, K']``; a two-site tensor is
``x[a, s1, s2, b]``.

* ``heff_apply``   two-site form of the matvec eq. mat_vec, contracted in the
                   order L.x -> W1 -> W2 -> R.
* ``env_left``     one update step of eq. env_L (contract one transfer tensor
                   G_j into the left environment).
* ``env_right``    one update step of eq. env_R.
* ``overlap_left`` / ``overlap_right``: the same without an operator (the
                   TT inner products of Section A.2).
* ``heff_grads``   partial derivatives of ``E = <x|H_eff|x>`` with respect to
                   every operand (each is the contraction with that operand
                   removed).

Sparse MPO cores are given as ``(A_idx, B_idx, ops)`` with ``ops[e]`` the
4x4 local operator ``W[A_idx[e], :, :, B_idx[e]]``.
"""
from __future__ import annotations

import numpy as np


def dense_core(Aidx, Bidx, ops, R_left, R_right):
    W = np.zeros((R_left, 4, 4, R_right))
    np.add.at(W, (Aidx, slice(None), slice(None), Bidx), ops)
    return W


def heff_apply(Lenv, W1, W2, Renv, x):
    """y[a',s1',s2',b'] = sum L[a',A,a] W1[A,s1',s1,B] W2[B,s2',s2,C] R[b',C,b] x[a,s1,s2,b]."""
    t1 = np.einsum("pAa,astb->pAstb", Lenv, x)
    t2 = np.einsum("AuwB,pAwtb->puBtb", W1, t1)
    t3 = np.einsum("BvtC,puBtb->puvCb", W2, t2)
    return np.einsum("qCb,puvCb->puvq", Renv, t3)


def heff_matrix(Lenv, W1, W2, Renv):
    """Explicit H_eff as a matrix on vec(x) (row-major x)."""
    rl, rr = Lenv.shape[0], Renv.shape[0]
    n = rl * 16 * rr
    M = np.einsum("pAa,AuwB,BvtC,qCb->puvqawtb", Lenv, W1, W2, Renv)
    return M.reshape(n, n)


def env_left(Lenv, Ubra, W, Uket):
    """L'[b',B,b] = sum L[a',A,a] Ubra[a',s',b'] W[A,s',s,B] Uket[a,s,b]."""
    t = np.einsum("pAa,asb->pAsb", Lenv, Uket)
    t = np.einsum("AusB,pAsb->puBb", W, t)
    return np.einsum("pud,puBb->dBb", Ubra, t)


def env_right(Renv, Ubra, W, Uket):
    """R'[a',A,a] = sum Ubra[a',s',b'] W[A,s',s,B] Uket[a,s,b] R[b',B,b]."""
    t = np.einsum("qBb,asb->qBas", Renv, Uket)
    t = np.einsum("AusB,qBas->qAau", W, t)
    return np.einsum("puq,qAau->pAa", Ubra, t)


def overlap_left(E, Ubra, Uket):
    return np.einsum("pa,psb,asc->bc", E, Ubra, Uket)


def overlap_right(E, Ubra, Uket):
    return np.einsum("bc,psb,asc->pa", E, Ubra, Uket)


def heff_grads(Lenv, W1, W2, Renv, x):
    """Energy E = <x|H_eff x> and its partial derivatives with respect to
    x, L, W1, W2 and R (no symmetry of H_eff assumed)."""
    y = heff_apply(Lenv, W1, W2, Renv, x)
    E = float(np.sum(x * y))
    # H^T x: the same contraction with bra and ket roles of every operand swapped
    LT = Lenv.transpose(2, 1, 0)
    RT = Renv.transpose(2, 1, 0)
    W1T = W1.transpose(0, 2, 1, 3)
    W2T = W2.transpose(0, 2, 1, 3)
    gx = y + heff_apply(LT, W1T, W2T, RT, x)
    # every gradient is the contraction with one operand removed, taken in
    # pairwise steps
    Rx = np.einsum("qCb,awtb->qCawt", Renv, x)
    W2Rx = np.einsum("BvtC,qCawt->qBvaw", W2, Rx)
    W1W2Rx = np.einsum("AuwB,qBvaw->qAuva", W1, W2Rx)
    gL = np.einsum("puvq,qAuva->pAa", x, W1W2Rx)
    Lx = np.einsum("pAa,awtb->pAwtb", Lenv, x)
    W1Lx = np.einsum("AuwB,pAwtb->puBtb", W1, Lx)
    W2W1Lx = np.einsum("BvtC,puBtb->puvCb", W2, W1Lx)
    gR = np.einsum("puvq,puvCb->qCb", x, W2W1Lx)
    W2R = np.einsum("BvtC,qCb->Bvtqb", W2, Renv)
    xW2R = np.einsum("puvq,Bvtqb->puBtb", x, W2R)
    gW1 = np.einsum("puBtb,pAwtb->AuwB", xW2R, Lx)
    xR = np.einsum("puvq,qCb->puvCb", x, Renv)
    gW2 = np.einsum("puvCb,puBtb->BvtC", xR, W1Lx)
    return E, gx, gL, gW1, gW2, gR


# ---------------------------------------------------------------------------
# sparse-core variants for sampled checks at full size
# ---------------------------------------------------------------------------

def _apply_sparse_left(T, Aidx, Bidx, ops, R_out, axis_site):
    """out[B, ...] = sum_e ops[e][s_out, s_in] T[A_e, ... s_in ...] with the site
    index at position ``axis_site`` of T[A]."""
    shp = list(T.shape)
    shp[0] = R_out
    out = np.zeros(shp)
    for e in range(len(Aidx)):
        blk = np.tensordot(ops[e], T[Aidx[e]], axes=([1], [axis_site - 1]))
        blk = np.moveaxis(blk, 0, axis_site - 1)
        out[Bidx[e]] += blk
    return out


def heff_rows(Lrows, x, W1s, W2s, R_m, R_r, Renv_cols):
    """Sampled matvec: ``y[a'_i, :, :, b'_j]`` for given rows ``Lrows[i] = L[a'_i]``
    (layout [A][a]) and ``Renv_cols[j] = R[b'_j]`` (layout [C][b]); W cores sparse.
    Returns an array [i, j, s1', s2']."""
    rl, _, _, rr = x.shape
    out = np.zeros((len(Lrows), len(Renv_cols), 4, 4))
    X = x.reshape(rl, -1)
    for i, Lr in enumerate(Lrows):
        T = (Lr @ X).reshape(Lr.shape[0], 4, 4, rr)
        T2 = _apply_sparse_left(T, *W1s, R_m, axis_site=1)
        T3 = _apply_sparse_left(T2, *W2s, R_r, axis_site=2)
        for j, Rc in enumerate(Renv_cols):
            out[i, j] = np.einsum("Cuvb,Cb->uv", T3, Rc)
    return out
