"""Environment-chain oracle: two-site DMRG and additive two-level DMRG at any size.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Where ``oracle.tt`` forms dense 4^L state vectors (exact but limited to
L <= 8), this module follows the same algorithms through tensor-train
contractions only, so it reaches the sizes of the bench workloads:

* environments (eq. env_L, eq. env_R) built site by site from the oracle's own
  MPO (``oracle.mpo``), one site update being: contract the ket core, apply
  the MPO core as a sparse matrix over (channel, local state), contract the
  bra core;
* the two-site effective operator (eq. mat_vec, two-site form) applied in the
  order L.x -> W1 -> W2 -> R, and its lowest eigenpair on the
  quantum-number-allowed entries of x by Lanczos (the local solver of the
  paper's experiments, Section 4) started from the current two-site tensor;
* Algorithm 2 (two-site branch, subdomains of Extension Two): the first
  block's right-to-left LQ sweep, one left-to-right sweep per subdomain over
  bonds (s_j, s_j+1) .. (e_j, e_j+1) (the last subdomain stops at
  (L-2, L-1)), the coarse matrices of eq. d_opt_lin_3/4 and eq. A_reduced as
  TT inner products and sandwiches <tau(U^i)|H|tau(U^j)> (Appendix A.2)
  contracted from the left over all sites, the coarse eigenproblem of
  ``oracle.tt.coarse_solve``, and Step 4 as TT rounding (right-to-left QR,
  left-to-right truncated SVD with the truncation rule of
  ``oracle.tt.truncation_keep``) of the textbook direct-sum tensor train of
  sum_j c_j tau(U^j);
* Algorithm 2, one-site branch: the one-site operator (eq. mat_vec) applied as
  L.x -> W -> R, subdomain j swept over sites s_j .. e_j with the
  orthogonalization step of Algorithm 1 (``oracle.tt.qr_left_core``) moving the
  centre right between micro-steps;
* the linear-system functional (eq. energy_lin): the micro-steps solve
  P^T A P w = P^T F by conjugate gradients on the same products, P^T F from the
  overlap environments of the iterate with F's TT; the coarse linear system over
  the normalised updates (``oracle.tt.coarse_solve_lin``), b_j = <U^j|F> by overlap
  chains;
* Algorithm 1 (two-site branch) with the same pieces.

Every dense step is a library matrix product or factorisation on plain
arrays; the MPO core is applied with ``scipy.sparse``.  Index conventions:
environment E[bra, channel, ket], MPO core W[A, s_out, s_in, B], core
U[a, s, b], two-site tensor x[a, s1, s2, b].
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import tt as T
from .lanczos import lanczos_lowest


# ---------------------------------------------------------------------------
# the MPO core as sparse matrices over (channel, local state)
# ---------------------------------------------------------------------------

@dataclass
class SiteOps:
    fw: sp.csr_matrix   # [(B, s_out), (A, s_in)] = W[A, s_out, s_in, B]
    bw: sp.csr_matrix   # [(A, s_out), (B, s_in)] = W[A, s_out, s_in, B]
    RA: int
    RB: int


_POOL = None


def spmm(M, D):
    """M @ D for a sparse M and a dense D, the columns of D split over threads
    (the sparse product runs outside the interpreter lock)."""
    global _POOL
    nthr = min(os.cpu_count() or 1, 16)
    if D.shape[1] < 4096 or nthr == 1:
        return M @ D
    if _POOL is None:
        _POOL = ThreadPoolExecutor(nthr)
    cuts = np.linspace(0, D.shape[1], nthr + 1).astype(int)
    parts = list(_POOL.map(lambda i: M @ np.ascontiguousarray(D[:, cuts[i]:cuts[i + 1]]), range(nthr)))
    return np.concatenate(parts, axis=1)


def site_ops(mpo, k) -> SiteOps:
    A, B, ops = mpo.cores[k]
    RA, RB = mpo.R[k], mpo.R[k + 1]
    e, so, si = np.nonzero(ops)
    val = ops[e, so, si]
    fw = sp.csr_matrix((val, (B[e] * 4 + so, A[e] * 4 + si)), shape=(RB * 4, RA * 4))
    bw = sp.csr_matrix((val, (A[e] * 4 + so, B[e] * 4 + si)), shape=(RA * 4, RB * 4))
    return SiteOps(fw, bw, RA, RB)


# ---------------------------------------------------------------------------
# contractions
# ---------------------------------------------------------------------------

def env_left(E, bra, W: SiteOps, ket):
    """E'[b', B, b] = sum E[a', A, a] bra[a', s', b'] W[A, s', s, B] ket[a, s, b]."""
    rbra, RA, rket = E.shape
    rb2, rk2 = bra.shape[2], ket.shape[2]
    t = (E.transpose(1, 0, 2).reshape(RA * rbra, rket) @ ket.reshape(rket, 4 * rk2)).reshape(RA, rbra, 4, rk2)
    t = t.transpose(0, 2, 1, 3).reshape(RA * 4, rbra * rk2)
    t = spmm(W.fw, t)                                   # [B s', a' b]
    t = t.reshape(W.RB, 4, rbra, rk2).transpose(0, 3, 2, 1).reshape(W.RB * rk2, rbra * 4)
    out = t @ bra.reshape(rbra * 4, rb2)                # [B b, b']
    return np.ascontiguousarray(out.reshape(W.RB, rk2, rb2).transpose(2, 0, 1))


def env_right(E, bra, W: SiteOps, ket):
    """E'[a', A, a] = sum bra[a', s', b'] W[A, s', s, B] ket[a, s, b] E[b', B, b]."""
    rbra2, RB, rket2 = E.shape
    rbra, rket = bra.shape[0], ket.shape[0]
    t = E.transpose(1, 0, 2).reshape(RB * rbra2, rket2) @ ket.reshape(rket * 4, rket2).T   # [B b', a s]
    t = t.reshape(RB, rbra2, rket, 4).transpose(0, 3, 1, 2).reshape(RB * 4, rbra2 * rket)
    t = spmm(W.bw, t)                                   # [A s', b' a]
    t = t.reshape(W.RA, 4, rbra2, rket).transpose(1, 2, 0, 3).reshape(4 * rbra2, W.RA * rket)
    out = bra.reshape(rbra, 4 * rbra2) @ t              # [a', A a]
    return out.reshape(rbra, W.RA, rket)


def overlap_left(E, bra, ket):
    """E'[b', b] = sum E[a', a] bra[a', s, b'] ket[a, s, b]."""
    t = (E @ ket.reshape(ket.shape[0], -1)).reshape(bra.shape[0] * 4, ket.shape[2])
    return bra.reshape(bra.shape[0] * 4, bra.shape[2]).T @ t


def overlap_right(E, bra, ket):
    """E'[a', a] = sum bra[a', s, b'] ket[a, s, b] E[b', b]."""
    t = ket.reshape(ket.shape[0] * 4, ket.shape[2]) @ E.T          # [a s, b']
    t = t.reshape(ket.shape[0], 4 * bra.shape[2])
    return bra.reshape(bra.shape[0], 4 * bra.shape[2]) @ t.T        # [a', a]


def heff_apply(Lenv, W1: SiteOps, W2: SiteOps, Renv, x):
    """y[a', s1', s2', b'] = sum L[a', A, a] W1[A, s1', s1, B] W2[B, s2', s2, C] R[b', C, b] x[a, s1, s2, b].
    The bra dimensions a', b' are those of the environments (a subset of bra rows of L
    gives exactly those rows of y)."""
    rl, rr = x.shape[0], x.shape[3]
    pl, pr = Lenv.shape[0], Renv.shape[0]
    RA, RC = W1.RA, W2.RB
    t = (Lenv.transpose(1, 0, 2).reshape(RA * pl, rl) @ x.reshape(rl, 16 * rr)).reshape(RA, pl, 4, 4, rr)
    t = t.transpose(0, 2, 1, 3, 4).reshape(RA * 4, pl * 4 * rr)         # [A s1, a' s2 b]
    t = spmm(W1.fw, t)                                                  # [B s1', a' s2 b]
    t = t.reshape(W1.RB, 4, pl, 4, rr).transpose(0, 3, 2, 1, 4).reshape(W1.RB * 4, pl * 4 * rr)
    t = spmm(W2.fw, t)                                                  # [C s2', a' s1' b]
    t = t.reshape(RC, 4, pl, 4, rr).transpose(2, 3, 1, 0, 4).reshape(pl * 16, RC * rr)
    y = t @ Renv.reshape(pr, RC * rr).T
    return y.reshape(pl, 4, 4, pr)


def heff1_apply(Lenv, W: SiteOps, Renv, x):
    """y[a', s', b'] = sum L[a', A, a] W[A, s', s, B] R[b', B, b] x[a, s, b] (one-site form)."""
    rl, rr = x.shape[0], x.shape[2]
    pl, pr = Lenv.shape[0], Renv.shape[0]
    RA, RB = W.RA, W.RB
    t = (Lenv.transpose(1, 0, 2).reshape(RA * pl, rl) @ x.reshape(rl, 4 * rr)).reshape(RA, pl, 4, rr)
    t = t.transpose(0, 2, 1, 3).reshape(RA * 4, pl * rr)               # [A s, a' b]
    t = spmm(W.fw, t)                                                  # [B s', a' b]
    t = t.reshape(RB, 4, pl, rr).transpose(2, 1, 0, 3).reshape(pl * 4, RB * rr)
    y = t @ Renv.reshape(pr, RB * rr).T
    return y.reshape(pl, 4, pr)


def chain_energy(mpo, ops, cores):
    """<U|H|U> / <U|U> by one left-to-right environment chain."""
    E = np.ones((1, 1, 1))
    N = np.ones((1, 1))
    for k, U in enumerate(cores):
        E = env_left(E, U, ops[k], U)
        N = overlap_left(N, U, U)
    return float(E[0, 0, 0] / N[0, 0])


def chain_sandwich(ops, bra, ket):
    """<bra|H|ket> and <bra|ket> (TT inner product and sandwich, Appendix A.2)."""
    E = np.ones((1, 1, 1))
    N = np.ones((1, 1))
    for k in range(len(bra)):
        E = env_left(E, bra[k], ops[k], ket[k])
        N = overlap_left(N, bra[k], ket[k])
    return float(E[0, 0, 0]), float(N[0, 0])


# ---------------------------------------------------------------------------
# local eigenproblem (micro-iteration)
# ---------------------------------------------------------------------------

def local_solve_k(Lenv, W1, W2, Renv, x0, ql, qr, K, tol=1e-12):
    """The K lowest eigenpairs of the two-site effective operator on the allowed
    entries (Extension One), by ARPACK's implicitly restarted Lanczos
    (scipy.sparse.linalg.eigsh), or dense eigh for small local spaces.  Returns a
    list of (theta, x) in increasing theta, and the number of products."""
    return _k_lowest(lambda z: heff_apply(Lenv, W1, W2, Renv, z), T.x_mask(ql, qr), x0, K, tol)


def local_solve1_k(Lenv, W, Renv, x0, ql, qr, K, tol=1e-12):
    """``local_solve_k`` for the one-site operator of ``heff1_apply``."""
    return _k_lowest(lambda z: heff1_apply(Lenv, W, Renv, z), T.x1_mask(ql, qr), x0, K, tol)


def _k_lowest(apply, m, x0, K, tol):
    from scipy.sparse.linalg import LinearOperator, eigsh

    dim = int(m.sum())
    count = [0]

    def mv(v):
        z = np.zeros(m.shape)
        z[m] = np.ravel(v)
        count[0] += 1
        return apply(z)[m]

    if dim <= 400:
        H = np.stack([mv(e) for e in np.eye(dim)], axis=1)
        w, v = np.linalg.eigh(0.5 * (H + H.T))
    else:
        start = x0[m] if np.any(x0[m]) else np.ones(dim)
        w, v = eigsh(LinearOperator((dim, dim), matvec=mv, dtype=np.float64), k=K, which="SA", v0=start, tol=tol,
                     ncv=max(4 * K, 24))
        o = np.argsort(w)
        w, v = w[o], v[:, o]
    out = []
    for q in range(min(K, w.size)):
        x = np.zeros(m.shape)
        x[m] = v[:, q] / np.linalg.norm(v[:, q])
        out.append((float(w[q]), x))
    return out, count[0]


def local_solve(Lenv, W1, W2, Renv, x0, ql, qr, tol=1e-11, maxiter=1000):
    """Lowest eigenpair of the two-site effective operator on the entries of x
    allowed by the bond charges (Lemma "DMRG micro-iterations for eigenvalue
    problems").  Returns (theta, x, matvecs)."""
    return _lowest(lambda z: heff_apply(Lenv, W1, W2, Renv, z), T.x_mask(ql, qr), x0, tol, maxiter)


def local_solve1(Lenv, W, Renv, x0, ql, qr, tol=1e-11, maxiter=1000):
    """``local_solve`` for the one-site operator of ``heff1_apply`` (x0, x: one core)."""
    return _lowest(lambda z: heff1_apply(Lenv, W, Renv, z), T.x1_mask(ql, qr), x0, tol, maxiter)


def _lowest(apply, m, x0, tol, maxiter):
    count = [0]

    def mv(v):
        z = np.zeros(m.shape)
        z[m] = v
        count[0] += 1
        return apply(z)[m]

    start = x0[m]
    if not np.any(start):
        start = np.ones(int(m.sum()))
    theta, u = lanczos_lowest(mv, start, tol=tol, maxiter=maxiter)
    x = np.zeros(m.shape)
    x[m] = u
    return float(theta), x, count[0]


# ---------------------------------------------------------------------------
# Algorithm 1 (two-site branch)
# ---------------------------------------------------------------------------

def dmrg2(mpo, cores, labels, chi, nsweeps=1, tol=1e-11, cutoff=1e-12, tau=1e-10):
    """Classical two-site DMRG from a left-orthogonal TT; returns the last Ritz
    value of every half sweep and the final TT."""
    L = mpo.L
    ops = [site_ops(mpo, k) for k in range(L)]
    labels = [q.copy() for q in labels]
    V, W = T.lq_sweep(cores, labels)
    cur = [W[0]] + [V[k] for k in range(1, L)]
    Le = [None] * (L + 1)
    Re = [None] * (L + 1)
    Le[0] = np.ones((1, 1, 1))
    Re[L] = np.ones((1, 1, 1))
    for k in range(L - 1, 1, -1):
        Re[k] = env_right(Re[k + 1], cur[k], ops[k], cur[k])
    energies = []
    for _ in range(nsweeps):
        for b in range(L - 1):
            x = np.einsum("asb,btc->astc", cur[b], cur[b + 1])
            theta, x, _ = local_solve(Le[b], ops[b], ops[b + 1], Re[b + 2], x, labels[b], labels[b + 2], tol)
            A, C, qn, _, _ = T.split_two_site(x, labels[b], labels[b + 2], chi, True, cutoff, tau)
            cur[b], cur[b + 1], labels[b + 1] = A, C, qn
            Le[b + 1] = env_left(Le[b], A, ops[b], A)
        energies.append(theta)
        for b in range(L - 2, -1, -1):
            x = np.einsum("asb,btc->astc", cur[b], cur[b + 1])
            theta, x, _ = local_solve(Le[b], ops[b], ops[b + 1], Re[b + 2], x, labels[b], labels[b + 2], tol)
            A, C, qn, _, _ = T.split_two_site(x, labels[b], labels[b + 2], chi, False, cutoff, tau)
            cur[b], cur[b + 1], labels[b + 1] = A, C, qn
            Re[b + 1] = env_right(Re[b + 2], C, ops[b + 1], C)
        energies.append(theta)
    return energies, cur, labels


# ---------------------------------------------------------------------------
# Step 4: direct sum and TT rounding
# ---------------------------------------------------------------------------

def tt_direct_sum(states, coef, labels_of):
    """Cores and labels of sum_j coef[j] * tau(states[j]) (block-diagonal
    interior cores, coefficients in the first core)."""
    L = len(states[0])
    cores, labels = [], []
    for k in range(L):
        rl = [st[k].shape[0] for st in states]
        rr = [st[k].shape[2] for st in states]
        if k == 0:
            C = np.concatenate([c * st[0] for c, st in zip(coef, states)], axis=2)
        elif k == L - 1:
            C = np.concatenate([st[k] for st in states], axis=0)
        else:
            C = np.zeros((sum(rl), 4, sum(rr)))
            i0 = j0 = 0
            for st, a, b in zip(states, rl, rr):
                C[i0:i0 + a, :, j0:j0 + b] = st[k]
                i0 += a
                j0 += b
        cores.append(C)
    for k in range(L + 1):
        if k == 0 or k == L:
            labels.append(labels_of[0][k].copy())
        else:
            labels.append(np.concatenate([lab[k] for lab in labels_of], axis=0))
    return cores, labels


def _groups(q):
    keys = {}
    for i, row in enumerate(map(tuple, q)):
        keys.setdefault(row, []).append(i)
    return {k: np.asarray(v) for k, v in keys.items()}


def right_orthogonalize(cores, labels):
    """Right-to-left sweep of charge-block QR factorisations (of the transposed
    unfoldings), so that cores 1..L-1 have orthonormal rows; bond sizes shrink
    to the rank bound min(rows, columns) of each block."""
    cores = [c.copy() for c in cores]
    labels = [q.copy() for q in labels]
    L = len(cores)
    for k in range(L - 1, 0, -1):
        U = cores[k]
        r, _, r2 = U.shape
        M = U.reshape(r, 4 * r2)
        col_q = (labels[k + 1][None, :, :] - T.SITE_Q[:, None, :]).reshape(-1, 2)
        rg, cg = _groups(labels[k]), _groups(col_q)
        newQ, newL, newlab = [], [], []
        for g in sorted(rg):
            rows = rg[g]
            cols = cg.get(g)
            if cols is None:
                continue
            q, rmat = np.linalg.qr(M[np.ix_(rows, cols)].T)     # block^T = q rmat
            kk = q.shape[1]
            Qb = np.zeros((kk, 4 * r2))
            Qb[:, cols] = q.T
            Lb = np.zeros((r, kk))
            Lb[rows, :] = rmat.T
            newQ.append(Qb)
            newL.append(Lb)
            newlab.extend([g] * kk)
        Qm = np.concatenate(newQ, axis=0)
        Lm = np.concatenate(newL, axis=1)
        cores[k] = Qm.reshape(-1, 4, r2)
        cores[k - 1] = np.einsum("asb,bc->asc", cores[k - 1], Lm)
        labels[k] = np.asarray(newlab, dtype=labels[k].dtype).reshape(-1, 2)
    return cores, labels


def tt_round(cores, labels, chi, cutoff=1e-12, tau=1e-10):
    """TT rounding: right orthogonalisation, then truncated charge-block SVDs
    from left to right (result left-orthogonal)."""
    cores, labels = right_orthogonalize(cores, labels)
    L = len(cores)
    for k in range(L - 1):
        U = cores[k]
        r, _, r2 = U.shape
        row_q = (labels[k][:, None, :] + T.SITE_Q[None, :, :]).reshape(-1, 2)
        Um, s, Vt, qn, _ = T.sector_svd(U.reshape(r * 4, r2), row_q, labels[k + 1], chi, cutoff, tau)
        cores[k] = Um.reshape(r, 4, -1)
        cores[k + 1] = np.einsum("ab,bsc->asc", s[:, None] * Vt, cores[k + 1])
        labels[k + 1] = qn.astype(labels[k + 1].dtype)
    return cores, labels


# ---------------------------------------------------------------------------
# Algorithm 2 (two-site branch, subdomains)
# ---------------------------------------------------------------------------

@dataclass
class ChainReport:
    E_before: float
    E_local: list
    matvecs: list
    S: np.ndarray
    A: np.ndarray
    lam: float
    c: np.ndarray
    rankS: int
    E_new: float
    cores: list
    labels: list
    states: list
    state_labels: list


def a2dmrg_sweep(mpo, cores, labels, chi, lengths, eps=1e-8, tol=1e-11, cutoff=1e-12, tau=1e-10, log=None,
                 n_eig=1, sites=2):
    """One global iteration of Algorithm 2 from a left-orthogonal TT
    (U_0..U_{L-2}, W_{L-1}).  Same readings as ``oracle.tt.a2dmrg_sweep``,
    including ``n_eig`` (Extension One at every subdomain's last micro-step) and
    ``sites`` (1: one-site micro-steps)."""
    L = mpo.L
    ops = [site_ops(mpo, k) for k in range(L)]
    cores = [c.copy() for c in cores]
    cores[-1] = cores[-1] / np.linalg.norm(cores[-1])
    E_before = chain_energy(mpo, ops, cores)
    V, W = T.lq_sweep(cores, labels)
    starts = T.subdomain_starts(lengths)
    # left environments of the left-orthogonal iterate, right ones of the right-orthogonal cores
    Le = [np.ones((1, 1, 1))]
    for k in range(max(starts)):
        Le.append(env_left(Le[k], cores[k], ops[k], cores[k]))
    Re = [None] * (L + 1)
    Re[L] = np.ones((1, 1, 1))
    # a one-site micro-step at site k reads Re[k + 1], a two-site one at (b, b + 1) Re[b + 2]
    kmin = 1 if sites == 1 else 2
    for k in range(L - 1, kmin - 1, -1):
        Re[k] = env_right(Re[k + 1], V[k], ops[k], V[k])
    states, state_labels = [cores], [labels]
    E_local, matvecs = [], []
    for j, s in enumerate(starts):
        e = s + lengths[j] - 1
        lab = [q.copy() for q in labels]
        cur = cores[:s] + [W[s]] + [V[k] for k in range(s + 1, L)]
        Lrun = Le[s]
        blast = min(e, L - 2)
        theta, nmv = 0.0, 0
        alts = []
        if sites == 1:
            for k in range(s, e + 1):
                if k == e and n_eig > 1:
                    pairs, nk = local_solve1_k(Lrun, ops[k], Re[k + 1], cur[k], lab[k], lab[k + 1], n_eig)
                    theta, x = pairs[0]
                    for _, xq in pairs[1:]:
                        alt = list(cur)
                        alt[k] = xq / np.linalg.norm(xq)
                        alts.append((alt, [q.copy() for q in lab]))
                else:
                    theta, x, nk = local_solve1(Lrun, ops[k], Re[k + 1], cur[k], lab[k], lab[k + 1], tol)
                nmv += nk
                if k < e:
                    Q, R = T.qr_left_core(x, lab[k], lab[k + 1])
                    cur[k], cur[k + 1] = Q, np.einsum("ab,bsc->asc", R, cur[k + 1])
                    Lrun = env_left(Lrun, Q, ops[k], Q)
                else:
                    cur[k] = x / np.linalg.norm(x)
                if log:
                    log(f"subdomain {j} site {k}: theta={theta:.12f} products={nk}")
            blast = -1  # no two-site micro-steps
        for b in range(s, blast + 1):
            x = np.einsum("asb,btc->astc", cur[b], cur[b + 1])
            if b == blast and n_eig > 1:
                pairs, k = local_solve_k(Lrun, ops[b], ops[b + 1], Re[b + 2], x, lab[b], lab[b + 2], n_eig)
                theta, x = pairs[0]
                for _, xq in pairs[1:]:
                    Aq, Cq, qq, _, _ = T.split_two_site(xq, lab[b], lab[b + 2], chi, True, cutoff, tau)
                    alt, alt_lab = list(cur), [q.copy() for q in lab]
                    alt[b], alt[b + 1], alt_lab[b + 1] = Aq, Cq / np.linalg.norm(Cq), qq
                    alts.append((alt, alt_lab))
            else:
                theta, x, k = local_solve(Lrun, ops[b], ops[b + 1], Re[b + 2], x, lab[b], lab[b + 2], tol)
            nmv += k
            A, C, qn, _, _ = T.split_two_site(x, lab[b], lab[b + 2], chi, True, cutoff, tau)
            cur[b], cur[b + 1], lab[b + 1] = A, C, qn
            if b < blast:
                Lrun = env_left(Lrun, A, ops[b], A)
            if log:
                log(f"subdomain {j} bond {b}: theta={theta:.12f} products={k}")
        if sites == 2 and s <= L - 2:
            cur[blast + 1] = cur[blast + 1] / np.linalg.norm(cur[blast + 1])
        states.append(cur)
        state_labels.append(lab)
        for alt, alt_lab in alts:
            states.append(alt)
            state_labels.append(alt_lab)
        E_local.append(theta)
        matvecs.append(nmv)
    n = len(states)
    S = np.zeros((n, n))
    A = np.zeros((n, n))
    for i in range(n):
        for jj in range(i, n):
            A[i, jj], S[i, jj] = chain_sandwich(ops, states[i], states[jj])
            A[jj, i], S[jj, i] = A[i, jj], S[i, jj]
    lam, c, rank = T.coarse_solve(S, A, eps)
    sc, sl = tt_direct_sum(states, c, state_labels)
    new_cores, new_labels = tt_round(sc, sl, chi, cutoff, tau)
    new_cores[-1] = new_cores[-1] / np.linalg.norm(new_cores[-1])
    E_new = chain_energy(mpo, ops, new_cores)
    return ChainReport(E_before, E_local, matvecs, S, A, lam, c, rank, E_new, new_cores, new_labels, states,
                       state_labels)


# ---------------------------------------------------------------------------
# linear-system functional (eq. energy_lin)
# ---------------------------------------------------------------------------

def conjugate_gradients(mv, b, x0, tol=1e-12, maxiter=1000):
    """Plain conjugate gradients for a symmetric positive definite operator: from x0
    until |b - A x| <= tol |b|.  Returns (x, products)."""
    x = x0.copy()
    r = b - mv(x)
    n = 1
    p = r.copy()
    rr = r @ r
    bn = np.linalg.norm(b)
    while np.sqrt(rr) > tol * bn and n < maxiter:
        q = mv(p)
        n += 1
        a = rr / (p @ q)
        x += a * p
        r -= a * q
        rr2 = r @ r
        p = r + (rr2 / rr) * p
        rr = rr2
    return x, n


def a2dmrg_lin_sweep(mpo, cores, labels, chi, lengths, f_cores, eps=1e-8, tol=1e-12, cutoff=1e-12, tau=1e-10,
                     sites=2, log=None):
    """One global iteration of Algorithm 2 for the linear-system functional with A the
    MPO operator: the readings of ``oracle.tt.a2dmrg_lin_sweep`` through environment
    chains.  ``cores``: left-orthogonal, the last core carrying the iterate's norm."""
    L = mpo.L
    ops = [site_ops(mpo, k) for k in range(L)]
    cores = [c.copy() for c in cores]

    def J_of(st):
        E = np.ones((1, 1, 1))
        N = np.ones((1, 1))
        G = np.ones((1, 1))
        for k in range(L):
            E = env_left(E, st[k], ops[k], st[k])
            G = overlap_left(G, st[k], f_cores[k])
        return float(0.5 * E[0, 0, 0] - G[0, 0])

    J_before = J_of(cores)
    V, W = T.lq_sweep(cores, labels)
    starts = T.subdomain_starts(lengths)
    Le = [np.ones((1, 1, 1))]
    Fe = [np.ones((1, 1))]
    for k in range(max(starts)):
        Le.append(env_left(Le[k], cores[k], ops[k], cores[k]))
        Fe.append(overlap_left(Fe[k], cores[k], f_cores[k]))
    Re = [None] * (L + 1)
    Fr = [None] * (L + 1)
    Re[L] = np.ones((1, 1, 1))
    Fr[L] = np.ones((1, 1))
    for k in range(L - 1, 0, -1):
        Re[k] = env_right(Re[k + 1], V[k], ops[k], V[k])
        Fr[k] = overlap_right(Fr[k + 1], V[k], f_cores[k])
    states, state_labels, E_local, matvecs = [cores], [labels], [], []
    for j, s in enumerate(starts):
        e = s + lengths[j] - 1
        lab = [q.copy() for q in labels]
        cur = cores[:s] + [W[s]] + [V[k] for k in range(s + 1, L)]
        Lrun, Frun = Le[s], Fe[s]
        theta, nmv = 0.0, 0
        if sites == 1:
            for k in range(s, e + 1):
                m = T.x1_mask(lab[k], lab[k + 1])
                rhs = np.einsum("ac,csd,bd->asb", Frun, f_cores[k], Fr[k + 1])[m]

                def mv(v, k=k, m=m):
                    z = np.zeros(m.shape)
                    z[m] = v
                    return heff1_apply(Lrun, ops[k], Re[k + 1], z)[m]

                w, n = conjugate_gradients(mv, rhs, cur[k][m], tol)
                nmv += n
                theta = float(0.5 * w @ mv(w) - rhs @ w)
                x = np.zeros(m.shape)
                x[m] = w
                if k < e:
                    Q, R = T.qr_left_core(x, lab[k], lab[k + 1])
                    cur[k], cur[k + 1] = Q, np.einsum("ab,bsc->asc", R, cur[k + 1])
                    Lrun = env_left(Lrun, Q, ops[k], Q)
                    Frun = overlap_left(Frun, Q, f_cores[k])
                else:
                    cur[k] = x
                if log:
                    log(f"subdomain {j} site {k}: J_loc={theta:.12f} products={n}")
        else:
            blast = min(e, L - 2)
            for b in range(s, blast + 1):
                m = T.x_mask(lab[b], lab[b + 2])
                fw = np.einsum("asb,btc->astc", f_cores[b], f_cores[b + 1])
                rhs = np.einsum("ac,cstd,bd->astb", Frun, fw, Fr[b + 2])[m]
                x0 = np.einsum("asb,btc->astc", cur[b], cur[b + 1])

                def mv(v, b=b, m=m):
                    z = np.zeros(m.shape)
                    z[m] = v
                    return heff_apply(Lrun, ops[b], ops[b + 1], Re[b + 2], z)[m]

                w, n = conjugate_gradients(mv, rhs, x0[m], tol)
                nmv += n
                theta = float(0.5 * w @ mv(w) - rhs @ w)
                x = np.zeros(m.shape)
                x[m] = w
                A_, C_, qn, _, _ = T.split_two_site(x, lab[b], lab[b + 2], chi, True, cutoff, tau)
                cur[b], cur[b + 1], lab[b + 1] = A_, C_, qn
                if b < blast:
                    Lrun = env_left(Lrun, A_, ops[b], A_)
                    Frun = overlap_left(Frun, A_, f_cores[b])
                if log:
                    log(f"subdomain {j} bond {b}: J_loc={theta:.12f} products={n}")
        states.append(cur)
        state_labels.append(lab)
        E_local.append(theta)
        matvecs.append(nmv)
    n = len(states)
    S = np.zeros((n, n))
    A = np.zeros((n, n))
    b = np.zeros(n)
    for i in range(n):
        G = np.ones((1, 1))
        for k in range(L):
            G = overlap_left(G, states[i][k], f_cores[k])
        b[i] = G[0, 0]
        for jj in range(i, n):
            A[i, jj], S[i, jj] = chain_sandwich(ops, states[i], states[jj])
            A[jj, i], S[jj, i] = A[i, jj], S[i, jj]
    d = 1.0 / np.sqrt(np.diag(S))
    S, A, b = S * np.outer(d, d), A * np.outer(d, d), b * d
    Jc, c, rank = T.coarse_solve_lin(S, A, b, eps)
    sc, sl = tt_direct_sum(states, c * d, state_labels)
    new_cores, new_labels = tt_round(sc, sl, chi, cutoff, tau)
    J_new = J_of(new_cores)
    rep = T.LinearReport(J_before, E_local, S, A, b, c, Jc, rank, J_new, new_cores, new_labels, states)
    rep.matvecs = matvecs
    return rep
