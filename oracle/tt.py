"""Tensor-train oracle: classical two-site DMRG and additive two-level DMRG.

Everything is written from the definitions of Sections 2-3 and works on dense
state vectors restricted to one (N, Sz) sector, so it is limited to small
``L`` (the Fock space has 4^L entries).

* TT contraction map tau (Definition "tensor train contraction mapping").
* Orthogonal decompositions (Definition "orthogonal tensor train
  decompositions"): left-orthogonalisation by sector-wise QR, the
  right-to-left LQ sweep of Algorithm 2 (first block).
* Two-site retraction P_{U,k,2} (Definition "retraction operators") formed as an
  explicit matrix; the micro-iteration S_{k,k+1} is the lowest eigenpair of
  ``P^T A P`` (Lemma "DMRG micro-iterations for eigenvalue problems").
* Truncated SVD per particle-number block (Section 3.2: truncation is applied
  on the individual non-zero blocks).  Truncation rule (the paper fixes only a
  tolerance): keep at most ``chi`` values, drop values below
  ``cutoff * s_max``; if the group of values within ``tau * s_max`` of the
  chi-th value straddles the cut, drop the whole group.
* Algorithm 1 (two-site branch) and Algorithm 2 (two-site branch) with the
  subdomain grouping of Extension Two: subdomain j = sites [s_j, e_j] is swept
  left to right over bonds (s_j, s_j+1) .. (e_j, e_j+1), the last subdomain
  stopping at (L-2, L-1), so every bond is optimised once per global iteration.
* Algorithm 2, one-site branch: the one-site retraction P_{U,k,1} as an explicit
  matrix, the micro-iteration S_k as the lowest eigenpair of ``P^T A P``, and
  subdomain j swept over sites s_j .. e_j with the orthogonalization step of
  Algorithm 1 (charge-block QR of the new core, its R factor carried into the
  next core) between micro-steps.
* Second-level problem (eq. d_opt_lin_3/4, eq. A_reduced and the
  rank-deficient branch eq. aux_eig_final_sym): coarse matrices from dense
  state vectors, eigen-decomposition of the overlap with relative threshold
  ``eps``, lowest eigenpair of the reduced pencil.
* Linear-system functional (eq. energy_lin, J(X) = 1/2 <X,AX> - <F,X> with A
  symmetric positive definite): the micro-step minimises J over the range of the
  retraction, i.e. solves P^T A P w = P^T F; the second level minimises J over the
  span of the updates, the linear system (X^T A X) y = X^T b with b_j = <F, U^j>
  on the numerical range of the overlap matrix (the same canonical
  orthogonalisation as the eigenvalue case).
* Compression (Step 4 of Algorithm 2): TT-SVD of the dense coarse solution
  with the same per-block truncation rule, which equals TT rounding of any
  exact TT representation of that vector.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fock
from .lanczos import lanczos_lowest

SITE_Q = np.array([(0, 0), (1, 1), (1, -1), (2, 0)], dtype=np.int64)


# ---------------------------------------------------------------------------
# contraction map and blocks
# ---------------------------------------------------------------------------

def contract_full(cores) -> np.ndarray:
    """tau(U): the full tensor, flattened in row-major site order."""
    M = cores[0].reshape(cores[0].shape[0] * 4, cores[0].shape[2])
    for U in cores[1:]:
        r, n, r2 = U.shape
        M = (M @ U.reshape(r, n * r2)).reshape(-1, r2)
    return M.reshape(-1)


def left_block(cores, k: int) -> np.ndarray:
    """Phi_L: contraction of cores 0..k-1 as a (4^k, r_k) matrix."""
    M = np.ones((1, 1))
    for U in cores[:k]:
        r, n, r2 = U.shape
        M = (M @ U.reshape(r, n * r2)).reshape(-1, r2)
    return M


def right_block(cores, k: int) -> np.ndarray:
    """Phi_R: contraction of cores k..L-1 as an (r_k, 4^(L-k)) matrix."""
    M = np.ones((1, 1))
    for U in reversed(cores[k:]):
        r, n, r2 = U.shape
        M = (U.reshape(r * n, r2) @ M).reshape(r, -1)
    return M


# ---------------------------------------------------------------------------
# QN-blocked linear algebra
# ---------------------------------------------------------------------------

def _groups(q):
    keys = {}
    for i, row in enumerate(map(tuple, q)):
        keys.setdefault(row, []).append(i)
    return {k: np.asarray(v) for k, v in keys.items()}


def truncation_keep(svals: np.ndarray, chi: int, cutoff: float, tau: float) -> int:
    """Number of leading values (sorted descending) kept by the truncation rule."""
    if svals.size == 0 or svals[0] <= 0.0:
        return 0
    smax = svals[0]
    n = int(np.sum(svals >= cutoff * smax))
    if n <= chi:
        return n
    ref = svals[chi - 1]
    grp = np.nonzero(np.abs(svals[:n] - ref) <= tau * smax)[0]
    if grp.size and grp.min() < chi and grp.max() >= chi:
        return int(grp.min())
    return chi


def sector_svd(M, row_q, col_q, chi, cutoff=1e-12, tau=1e-10):
    """Truncated SVD of a QN-block matrix.  Returns ``(U, s, Vt, q_new, discarded)``
    with the new bond ordered by charge, then by decreasing singular value."""
    rg, cg = _groups(row_q), _groups(col_q)
    trip = []
    for g, rows in rg.items():
        cols = cg.get(g)
        if cols is None:
            continue
        u, s, vt = np.linalg.svd(M[np.ix_(rows, cols)], full_matrices=False)
        for i in range(s.size):
            trip.append((s[i], g, rows, cols, u[:, i], vt[i]))
    trip.sort(key=lambda t: (-t[0], t[1]))
    allsv = np.array([t[0] for t in trip])
    keep = truncation_keep(allsv, chi, cutoff, tau)
    kept = trip[:keep]
    discarded = float(np.sum(allsv[keep:] ** 2))
    kept.sort(key=lambda t: (t[1], -t[0]))
    U = np.zeros((M.shape[0], keep))
    Vt = np.zeros((keep, M.shape[1]))
    s = np.zeros(keep)
    q_new = np.zeros((keep, 2), dtype=np.int64)
    for j, (sv, g, rows, cols, u, v) in enumerate(kept):
        U[rows, j] = u
        Vt[j, cols] = v
        s[j] = sv
        q_new[j] = g
    return U, s, Vt, q_new, discarded


def split_two_site(x, ql, qr, chi, left_normal=True, cutoff=1e-12, tau=1e-10):
    """Split a two-site tensor x[a,s1,s2,b] by the truncated block SVD.
    ``left_normal``: (N, Sigma V^T); otherwise (U Sigma, V^T)."""
    rl, _, _, rr = x.shape
    M = x.reshape(rl * 4, 4 * rr)
    row_q = (ql[:, None, :] + SITE_Q[None, :, :]).reshape(-1, 2)
    col_q = (qr[None, :, :] - SITE_Q[:, None, :]).reshape(-1, 2)
    U, s, Vt, qn, disc = sector_svd(M, row_q, col_q, chi, cutoff, tau)
    k = s.size
    if left_normal:
        A = U.reshape(rl, 4, k)
        C = (s[:, None] * Vt).reshape(k, 4, rr)
    else:
        A = (U * s[None, :]).reshape(rl, 4, k)
        C = Vt.reshape(k, 4, rr)
    return A, C, qn, s, disc


def _block_qr(M, row_q, col_q):
    """M = Q R per charge block with Q having orthonormal columns."""
    Q = np.zeros_like(M)
    R = np.zeros((M.shape[1], M.shape[1]))
    rg, cg = _groups(row_q), _groups(col_q)
    for g, cols in cg.items():
        rows = rg.get(g)
        if rows is None or rows.size < cols.size:
            raise ValueError("rank-deficient block in QR")
        q, r = np.linalg.qr(M[np.ix_(rows, cols)])
        Q[np.ix_(rows, cols)] = q
        R[np.ix_(cols, cols)] = r
    return Q, R


def left_orthogonalize(cores, labels):
    """Sector-wise QR sweep left to right; returns a left-orthogonal TT whose last
    core carries the (unnormalised) norm."""
    cores = [c.copy() for c in cores]
    for k in range(len(cores) - 1):
        U = cores[k]
        r, n, r2 = U.shape
        row_q = (labels[k][:, None, :] + SITE_Q[None, :, :]).reshape(-1, 2)
        Q, R = _block_qr(U.reshape(r * n, r2), row_q, labels[k + 1])
        cores[k] = Q.reshape(r, n, r2)
        cores[k + 1] = np.einsum("ab,bsc->asc", R, cores[k + 1])
    return cores


def lq_sweep(cores, labels):
    """First block of Algorithm 2: from a left-orthogonal TT (U_0..U_{L-2}, W_{L-1})
    produce the right-orthogonal cores V_k (k >= 1) and the centres W_k, so that
    (U_0..U_{k-1}, W_k, V_{k+1}..V_{L-1}) is the k-orthogonal copy."""
    L = len(cores)
    V = [None] * L
    W = [None] * L
    W[L - 1] = cores[L - 1].copy()
    for k in range(L - 1, 0, -1):
        r, n, r2 = W[k].shape
        col_q = (labels[k + 1][None, :, :] - SITE_Q[:, None, :]).reshape(-1, 2)
        Mt = W[k].reshape(r, n * r2).T
        Q, R = _block_qr(Mt, col_q, labels[k])
        V[k] = Q.T.reshape(r, n, r2)
        W[k - 1] = np.einsum("asb,cb->asc", cores[k - 1], R)
    return V, W


# ---------------------------------------------------------------------------
# retraction and the local eigenproblem
# ---------------------------------------------------------------------------

def x_mask(ql, qr) -> np.ndarray:
    tot = ql[:, None, None, None, :] + SITE_Q[None, :, None, None, :] + SITE_Q[None, None, :, None, :]
    return np.all(tot == qr[None, None, None, :, :], axis=-1)


def x1_mask(ql, qr) -> np.ndarray:
    """Allowed entries q(a) + q(s) = q(b) of one core."""
    tot = ql[:, None, None, :] + SITE_Q[None, :, None, :]
    return np.all(tot == qr[None, None, :, :], axis=-1)


def qr_left_core(x, ql, qr):
    """Orthogonalization step of Algorithm 1 (one-site branch): x[a, s, b] = Q R with Q
    left-orthogonal (charge-block QR of the (a s) x b unfolding); returns (Q, R)."""
    r, n, r2 = x.shape
    row_q = (ql[:, None, :] + SITE_Q[None, :, :]).reshape(-1, 2)
    Q, R = _block_qr(x.reshape(r * n, r2), row_q, qr)
    return Q.reshape(r, n, r2), R


class Problem:
    """Hamiltonian restricted to the target sector plus the index maps needed
    to move between dense vectors and tensor-train pieces."""

    def __init__(self, h, B, n_elec, two_sz=0):
        self.L = h.shape[0]
        self.n_elec = n_elec
        self.two_sz = two_sz
        self.states = fock.sector_states(self.L, n_elec, two_sz)
        self.tidx = fock.tensor_index(self.states, self.L)
        self.H = fock.hamiltonian(h, B, self.states, dense=True)

    def to_sector(self, full):
        return full[self.tidx]

    def energy(self, cores):
        y = self.to_sector(contract_full(cores))
        return float(y @ self.H @ y / (y @ y))

    def retraction(self, cores, k, ql, qr):
        """Explicit two-site retraction restricted to the sector rows and to the
        QN-allowed columns of x.  Returns (P, allowed_mask)."""
        L = self.L
        PhiL = left_block(cores, k)
        PhiR = right_block(cores, k + 2)
        nr = 4 ** (L - k - 2)
        il = self.tidx // (16 * nr)
        s12 = (self.tidx // nr) % 16
        ir = self.tidx % nr
        m = x_mask(ql, qr)
        a_i, s1_i, s2_i, b_i = np.nonzero(m)
        cs12 = s1_i * 4 + s2_i
        P = np.zeros((self.tidx.size, a_i.size))
        for v in range(16):
            rows = np.nonzero(s12 == v)[0]
            cols = np.nonzero(cs12 == v)[0]
            if rows.size and cols.size:
                P[np.ix_(rows, cols)] = PhiL[il[rows][:, None], a_i[cols][None, :]] * PhiR[b_i[cols][None, :], ir[rows][:, None]]
        return P, m

    def retraction1(self, cores, k, ql, qr):
        """Explicit one-site retraction P_{U,k,1} (cores 0..k-1 and k+1..L-1 of
        ``cores``) restricted to the sector rows and the allowed entries of the core."""
        L = self.L
        PhiL = left_block(cores, k)
        PhiR = right_block(cores, k + 1)
        nr = 4 ** (L - k - 1)
        il = self.tidx // (4 * nr)
        sv = (self.tidx // nr) % 4
        ir = self.tidx % nr
        m = x1_mask(ql, qr)
        a_i, s_i, b_i = np.nonzero(m)
        P = np.zeros((self.tidx.size, a_i.size))
        for v in range(4):
            rows = np.nonzero(sv == v)[0]
            cols = np.nonzero(s_i == v)[0]
            if rows.size and cols.size:
                P[np.ix_(rows, cols)] = PhiL[il[rows][:, None], a_i[cols][None, :]] * PhiR[b_i[cols][None, :], ir[rows][:, None]]
        return P, m

    def local_solve1_k(self, cores, k, ql, qr, K=1):
        """Micro-iteration S_k (one-site): the K lowest eigenpairs of P^T H P with the
        one-site retraction (dense eigensolver); unit eigenvectors as cores."""
        P, m = self.retraction1(cores, k, ql, qr)
        Heff = P.T @ self.H @ P
        w, v = np.linalg.eigh(0.5 * (Heff + Heff.T))
        out = []
        for q in range(min(K, w.size)):
            x = np.zeros(m.shape)
            x[m] = v[:, q]
            out.append((float(w[q]), x))
        return out

    def local_solve_lin(self, cores, k, ql, qr, f, sites=2):
        """Micro-step of the linear-system functional: w = (P^T A P)^{-1} P^T f with the
        two-site (or one-site) retraction; returns (1/2 w.P^T A P w - w.P^T f, w as a
        tensor)."""
        P, m = self.retraction(cores, k, ql, qr) if sites == 2 else self.retraction1(cores, k, ql, qr)
        Ap = P.T @ self.H @ P
        bp = P.T @ f
        w = np.linalg.solve(0.5 * (Ap + Ap.T), bp)
        x = np.zeros(m.shape)
        x[m] = w
        return float(0.5 * w @ Ap @ w - bp @ w), x

    def local_solve(self, cores, k, ql, qr, x0=None, tol=1e-12, dense_limit=3000):
        """Micro-iteration S_{k,k+1}: lowest eigenpair of P^T H P."""
        P, m = self.retraction(cores, k, ql, qr)
        n = P.shape[1]
        if n <= dense_limit:
            Heff = P.T @ self.H @ P
            w, v = np.linalg.eigh(0.5 * (Heff + Heff.T))
            theta, u = w[0], v[:, 0]
        else:
            HP = self.H @ P
            start = x0[m] if x0 is not None else np.ones(n)
            theta, u = lanczos_lowest(lambda z: P.T @ (HP @ z), start, tol=tol)
        x = np.zeros(m.shape)
        x[m] = u
        return float(theta), x

    def local_solve_k(self, cores, k, ql, qr, K):
        """The K lowest eigenpairs of P^T H P (Extension One); dense eigensolver."""
        P, m = self.retraction(cores, k, ql, qr)
        Heff = P.T @ self.H @ P
        w, v = np.linalg.eigh(0.5 * (Heff + Heff.T))
        out = []
        for q in range(min(K, w.size)):
            x = np.zeros(m.shape)
            x[m] = v[:, q]
            out.append((float(w[q]), x))
        return out


# ---------------------------------------------------------------------------
# Algorithm 1 (two-site) and Algorithm 2 (two-site, subdomain grouping)
# ---------------------------------------------------------------------------

def two_site(cores, k):
    return np.einsum("asb,btc->astc", cores[k], cores[k + 1])


def dmrg2(prob: Problem, cores, labels, chi, nsweeps=2, cutoff=1e-12, tau=1e-10):
    """Classical two-site DMRG (Algorithm 1, two-site branch), starting from a
    left-orthogonal TT which is first brought to right-orthogonal form.
    Returns the list of half-sweep energies and the final TT."""
    L = prob.L
    labels = [q.copy() for q in labels]
    V, W = lq_sweep(cores, labels)
    cur = [W[0]] + [V[k] for k in range(1, L)]
    energies = []
    for _ in range(nsweeps):
        for k in range(L - 1):
            theta, x = prob.local_solve(cur, k, labels[k], labels[k + 2])
            A, C, qn, _, _ = split_two_site(x, labels[k], labels[k + 2], chi, True, cutoff, tau)
            cur[k], cur[k + 1], labels[k + 1] = A, C, qn
        energies.append(theta)
        for k in range(L - 2, -1, -1):
            theta, x = prob.local_solve(cur, k, labels[k], labels[k + 2])
            A, C, qn, _, _ = split_two_site(x, labels[k], labels[k + 2], chi, False, cutoff, tau)
            cur[k], cur[k + 1], labels[k + 1] = A, C, qn
        energies.append(theta)
    return energies, cur, labels


def subdomain_starts(lengths):
    s = [0]
    for m in lengths[:-1]:
        s.append(s[-1] + m)
    return s


@dataclass
class SweepReport:
    E_local: list
    S: np.ndarray
    A: np.ndarray
    lam: float
    c: np.ndarray
    rankS: int
    E_new: float
    cores: list
    labels: list
    states: list = field(default_factory=list)


def coarse_solve(S, A, eps=1e-8):
    """Second-level problem: lowest eigenpair of the pencil (A, S) on the
    numerical range of S (eigenvalues of S below eps*max dropped)."""
    w, V = np.linalg.eigh(S)
    keep = w >= eps * w.max()
    X = V[:, keep] / np.sqrt(w[keep])[None, :]
    At = X.T @ A @ X
    lam, B = np.linalg.eigh(0.5 * (At + At.T))
    c = X @ B[:, 0]
    i = int(np.argmax(np.abs(c)))
    if c[i] < 0:
        c = -c
    return float(lam[0]), c, int(keep.sum())


def tt_svd(prob: Problem, y_sector, chi, cutoff=1e-12, tau=1e-10):
    """Left-orthogonal TT of a sector vector by sequential block SVDs."""
    L = prob.L
    full = np.zeros(4**L)
    full[prob.tidx] = y_sector
    target = np.array([prob.n_elec, prob.two_sz])
    ql = np.zeros((1, 2), dtype=np.int64)
    rem = full.reshape(1, -1)
    cores, labels = [], [ql]
    for k in range(L - 1):
        r = rem.shape[0]
        nright = 4 ** (L - k - 1)
        M = rem.reshape(r * 4, nright)
        row_q = (ql[:, None, :] + SITE_Q[None, :, :]).reshape(-1, 2)
        digits = np.arange(nright)
        cq = np.zeros((nright, 2), dtype=np.int64)
        for _ in range(L - k - 1):
            cq += SITE_Q[digits % 4]
            digits //= 4
        col_q = target[None, :] - cq
        U, s, Vt, qn, _ = sector_svd(M, row_q, col_q, chi, cutoff, tau)
        cores.append(U.reshape(r, 4, -1))
        labels.append(qn)
        rem = s[:, None] * Vt
        ql = qn
    cores.append(rem.reshape(rem.shape[0], 4, 1))
    labels.append(target[None, :].copy())
    return cores, labels


def a2dmrg_sweep(prob: Problem, cores, labels, chi, lengths, eps=1e-8, cutoff=1e-12, tau=1e-10, n_eig=1, sites=2):
    """One global iteration of Algorithm 2 (two-site, or one-site with ``sites=1``)
    with subdomains.

    ``cores`` must be left-orthogonal (U_0..U_{L-2}, W_{L-1}).  Returns a
    ``SweepReport`` with the local energies, the coarse matrices, the coarse
    eigenpair and the compressed next iterate (left-orthogonal, normalised).

    ``n_eig`` > 1: Extension One of the Remark on extensions of Algorithm 2, read
    for subdomains: the last micro-step of every subdomain keeps its ``n_eig``
    lowest eigenvectors, each giving an updated TT (coarse states ordered by
    subdomain, the lowest eigenvector's first).

    ``sites=1``: one-site micro-steps at sites s_j .. e_j of subdomain j, each followed
    (but the last) by the orthogonalization step that moves the centre right; the
    update is (U_0..U_{s-1}, Q_s..Q_{e-1}, x_e, V_{e+1}..V_{L-1}) with unit x_e, and
    its bond dimensions are those of the iterate.
    """
    L = prob.L
    norm0 = np.sqrt(np.sum(contract_full(cores) ** 2))
    cores = [c.copy() for c in cores]
    cores[-1] = cores[-1] / norm0
    V, W = lq_sweep(cores, labels)
    starts = subdomain_starts(lengths)
    states = [cores]
    E_local = []
    for j, s in enumerate(starts):
        e = s + lengths[j] - 1
        lab = [q.copy() for q in labels]
        cur = cores[:s] + [W[s]] + [V[k] for k in range(s + 1, L)]
        theta = None
        alts = []
        if sites == 1:
            for k in range(s, e + 1):
                pairs = prob.local_solve1_k(cur, k, lab[k], lab[k + 1], n_eig if k == e else 1)
                theta, x = pairs[0]
                if k < e:
                    cur[k], R = qr_left_core(x, lab[k], lab[k + 1])
                    cur[k + 1] = np.einsum("ab,bsc->asc", R, cur[k + 1])
                else:
                    for _, xq in pairs[1:]:
                        alt = list(cur)
                        alt[k] = xq / np.linalg.norm(xq)
                        alts.append(alt)
                    cur[k] = x / np.linalg.norm(x)
            states.append(cur)
            states.extend(alts)
            E_local.append(theta)
            continue
        blast = min(e, L - 2)
        for b in range(s, blast + 1):
            if b == blast and n_eig > 1:
                pairs = prob.local_solve_k(cur, b, lab[b], lab[b + 2], n_eig)
                theta, x = pairs[0]
                for _, xq in pairs[1:]:
                    A, C, qn, _, _ = split_two_site(xq, lab[b], lab[b + 2], chi, True, cutoff, tau)
                    alt = list(cur)
                    alt[b], alt[b + 1] = A, C / np.linalg.norm(C)
                    alts.append(alt)
            else:
                theta, x = prob.local_solve(cur, b, lab[b], lab[b + 2])
            A, C, qn, _, _ = split_two_site(x, lab[b], lab[b + 2], chi, True, cutoff, tau)
            cur[b], cur[b + 1], lab[b + 1] = A, C, qn
        last = blast + 1
        cur[last] = cur[last] / np.linalg.norm(cur[last])
        states.append(cur)
        states.extend(alts)
        E_local.append(theta)
    Y = np.stack([prob.to_sector(contract_full(st)) for st in states], axis=1)
    S = Y.T @ Y
    A = Y.T @ prob.H @ Y
    lam, c, rank = coarse_solve(S, A, eps)
    y = Y @ c
    new_cores, new_labels = tt_svd(prob, y, chi, cutoff, tau)
    nrm = np.sqrt(np.sum(contract_full(new_cores) ** 2))
    new_cores[-1] = new_cores[-1] / nrm
    E_new = prob.energy(new_cores)
    return SweepReport(E_local, S, A, lam, c, rank, E_new, new_cores, new_labels, states)


@dataclass
class LinearReport:
    J_before: float
    E_local: list
    S: np.ndarray
    A: np.ndarray
    b: np.ndarray
    c: np.ndarray
    J_coarse: float
    rankS: int
    J_new: float
    cores: list
    labels: list
    states: list


def coarse_solve_lin(S, A, b, eps=1e-8):
    """Second level of the linear-system functional: minimise 1/2 c.Ac - b.c over the
    numerical range of S (eigenvalues of S below eps*max dropped)."""
    w, V = np.linalg.eigh(S)
    keep = w >= eps * w.max()
    X = V[:, keep] / np.sqrt(w[keep])[None, :]
    At = X.T @ A @ X
    y = np.linalg.solve(0.5 * (At + At.T), X.T @ b)
    c = X @ y
    return float(0.5 * c @ A @ c - b @ c), c, int(keep.sum())


def a2dmrg_lin_sweep(prob: Problem, cores, labels, chi, lengths, f_cores, eps=1e-8, cutoff=1e-12, tau=1e-10,
                     sites=2):
    """One global iteration of Algorithm 2 for the linear-system functional, A = prob.H.

    ``cores``: left-orthogonal (U_0..U_{L-2}, W_{L-1}), W_{L-1} carrying the norm of the
    iterate X (not normalised: J depends on it); ``f_cores``: the TT of F.  The updates
    are the TTs of the micro-step solutions (two-site: split by the truncated SVD with
    the singular values on the right; one-site: QR moves); the coarse problem is posed
    on the normalised states (S with unit diagonal; c refers to them), and the
    combination is compressed by TT-SVD without normalisation."""
    L = prob.L
    f = prob.to_sector(contract_full(f_cores))
    V, W = lq_sweep(cores, labels)
    starts = subdomain_starts(lengths)
    states = [[c.copy() for c in cores]]
    E_local = []
    for j, s in enumerate(starts):
        e = s + lengths[j] - 1
        lab = [q.copy() for q in labels]
        cur = cores[:s] + [W[s]] + [V[k] for k in range(s + 1, L)]
        if sites == 1:
            for k in range(s, e + 1):
                theta, x = prob.local_solve_lin(cur, k, lab[k], lab[k + 1], f, sites=1)
                if k < e:
                    cur[k], R = qr_left_core(x, lab[k], lab[k + 1])
                    cur[k + 1] = np.einsum("ab,bsc->asc", R, cur[k + 1])
                else:
                    cur[k] = x
        else:
            blast = min(e, L - 2)
            theta = 0.0
            for b in range(s, blast + 1):
                theta, x = prob.local_solve_lin(cur, b, lab[b], lab[b + 2], f)
                A, C, qn, _, _ = split_two_site(x, lab[b], lab[b + 2], chi, True, cutoff, tau)
                cur[b], cur[b + 1], lab[b + 1] = A, C, qn
        states.append(cur)
        E_local.append(theta)
    Y = np.stack([prob.to_sector(contract_full(st)) for st in states], axis=1)
    x0 = Y[:, 0]
    J_before = float(0.5 * x0 @ prob.H @ x0 - f @ x0)
    # the coarse states are normalised (the span is unchanged, and the eps threshold of
    # the rank-deficient branch then does not depend on the states' scales)
    Y = Y / np.linalg.norm(Y, axis=0)[None, :]
    S = Y.T @ Y
    A = Y.T @ prob.H @ Y
    b = Y.T @ f
    Jc, c, rank = coarse_solve_lin(S, A, b, eps)
    y = Y @ c
    new_cores, new_labels = tt_svd(prob, y, chi, cutoff, tau)
    yn = prob.to_sector(contract_full(new_cores))
    J_new = float(0.5 * yn @ prob.H @ yn - f @ yn)
    return LinearReport(J_before, E_local, S, A, b, c, Jc, rank, J_new, new_cores, new_labels, states)
