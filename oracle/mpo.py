"""Matrix product operator of the electronic Hamiltonian, built for the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Written independently of
the library's own MPO builder: only its output (an MPO of the same operator)
is comparable, never its code.

The operator is the Hamiltonian of Section 3.2 in chemists' notation,

    H = sum_pq h_pq sum_s a+_ps a_qs
      + 1/2 sum_pqrs (pq|rs) sum_st a+_ps a+_rt a_st a_qs ,

(pq|rs) = sum_k B_k[p,q] B_k[r,s], written as a list of terms, each a
coefficient times a product of creation/annihilation operators.

Construction (the paper defers the MPO to the literature, eq. MPO):

* Every fermion operator is, in the Jordan-Wigner representation of
  ``oracle.fock`` (spin orbitals 0a,0b,1a,1b,..., local basis index
  n_a + 2 n_b), a Kronecker product of 4x4 site factors: the parity
  P = (-1)^n on every site left of its orbital, the local ladder operator on
  its site, the identity to the right.  A product of such operators is
  therefore the Kronecker product of the site-wise products of their
  factors, taken in operator order.  No reordering sign is needed.
* Each site factor is stored normalised (first non-zero entry positive) with
  its sign moved into the term's coefficient, so equal operator strings get
  equal keys.
* At the cut after ``l`` sites a term has n_L operators on the left and n_R on
  the right.  Its channel is labelled by its left factor string when
  n_L < n_R, or n_L == n_R and l <= L//2, and by its right factor string
  otherwise.  The labelling moves from left to right strings exactly once
  along the chain, and the coefficient is applied on that transition.
  Transitions inside the left (right) labelling only append a factor to the
  string and are shared by all terms with that string.

The bond dimension that results is 2 + 4L + 8m^2 - 2m with m = min(l, L-l)
(identity and completed strings, single operators on either side, and pairs
on the smaller side); the tests check this count and that the contracted MPO
equals the Fock-space matrix of ``oracle.fock``.

Output: per site ``k`` the sparse entries ``(A[e], B[e], ops[e])`` with
``ops[e] = W_k[A[e], :, :, B[e]]`` (row = output state), and the bond
dimensions ``R[0..L]``.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

# Jordan-Wigner site factors; rows = output state, columns = input state
PAR = np.diag([1.0, -1.0, -1.0, 1.0])
ID4 = np.eye(4)
# creation of an alpha electron: |0> -> |up>, |dn> -> |updn> (no other orbital
# of this site precedes alpha, so no sign inside the site)
CDAG_A = np.zeros((4, 4))
CDAG_A[1, 0] = 1.0
CDAG_A[3, 2] = 1.0
# creation of a beta electron: |0> -> |dn>, |up> -> |updn> with the sign of the
# alpha electron it passes
CDAG_B = np.zeros((4, 4))
CDAG_B[2, 0] = 1.0
CDAG_B[3, 1] = -1.0
LADDER = {(0, True): CDAG_A, (1, True): CDAG_B, (0, False): CDAG_A.T, (1, False): CDAG_B.T}


@dataclass
class OracleMPO:
    L: int
    R: list      # bond dimensions, R[0] = R[L] = 1
    cores: list  # per site (A int64 [nnz], B int64 [nnz], ops float64 [nnz, 4, 4])

    def dense_core(self, k):
        A, B, ops = self.cores[k]
        W = np.zeros((self.R[k], 4, 4, self.R[k + 1]))
        np.add.at(W, (A, slice(None), slice(None), B), ops)
        return W


def hamiltonian_terms(h, B):
    """The terms of H: list of (coefficient, ((spin orbital, is_creation), ...))
    in the written operator order."""
    L = h.shape[0]
    eri = np.einsum("kpq,krs->pqrs", B, B)
    terms = []
    for p, q in itertools.product(range(L), repeat=2):
        if h[p, q] != 0.0:
            for s in (0, 1):
                terms.append((float(h[p, q]), ((2 * p + s, True), (2 * q + s, False))))
    for p, q, r, t in itertools.product(range(L), repeat=4):
        v = eri[p, q, r, t]
        if v == 0.0:
            continue
        for s, u in itertools.product((0, 1), repeat=2):
            if (p, s) == (r, u) or (t, u) == (q, s):
                continue  # a+_i a+_i = a_i a_i = 0
            ops = ((2 * p + s, True), (2 * r + u, True), (2 * t + u, False), (2 * q + s, False))
            terms.append((0.5 * float(v), ops))
    return terms


class _FactorTable:
    """Dictionary of normalised 4x4 site factors: id <-> matrix."""

    def __init__(self):
        self.mats = []
        self.index = {}

    def key(self, M):
        """(id, sign) with M = sign * mats[id]; None for the zero matrix."""
        flat = M.reshape(-1)
        nz = np.nonzero(flat)[0]
        if nz.size == 0:
            return None
        sign = 1.0 if flat[nz[0]] > 0 else -1.0
        N = sign * M
        b = (np.round(N, 12) + 0.0).tobytes()  # + 0.0 turns -0.0 into 0.0
        i = self.index.get(b)
        if i is None:
            i = len(self.mats)
            self.index[b] = i
            self.mats.append(N.copy())
        return i, sign


def build_mpo(h, B) -> OracleMPO:
    L = h.shape[0]
    half = L // 2
    table = _FactorTable()
    id_I = table.key(ID4)[0]
    id_P = table.key(PAR)[0]
    Lset = [dict() for _ in range(L + 1)]   # cut -> {left string: index}
    Rset = [dict() for _ in range(L + 1)]   # cut -> {right string: index}
    shared = [dict() for _ in range(L)]     # site -> {(A key, B key, side): factor id}
    switch = [dict() for _ in range(L)]     # site -> {(left key, right key): summed 4x4}
    for coef, ops in hamiltonian_terms(h, B):
        sites = [so // 2 for so, _ in ops]
        occupied = sorted(set(sites))
        ids = []
        sign = 1.0
        zero = False
        for i in range(L):
            if i not in occupied:
                # parity from every operator whose orbital lies right of site i
                nright = sum(1 for s in sites if s > i)
                ids.append(id_P if nright % 2 else id_I)
                continue
            M = ID4
            for (so, cre), s in zip(ops, sites):
                if s > i:
                    F = PAR
                elif s == i:
                    F = LADDER[(so % 2, cre)]
                else:
                    F = ID4
                M = M @ F
            k = table.key(M)
            if k is None:
                zero = True
                break
            ids.append(k[0])
            sign *= k[1]
        if zero:
            continue
        ids = tuple(ids)
        nops = len(ops)

        def left_labelled(l):
            nl = sum(1 for s in sites if s < l)
            nr = nops - nl
            return nl < nr or (nl == nr and l <= half)

        # switch site: the last cut with a left label is i, the next (i + 1) has a right label
        i_sw = max(l for l in range(L + 1) if left_labelled(l))
        # left strings at cuts 0..i_sw, with their appending transitions
        for l in range(i_sw, -1, -1):
            key = ids[:l]
            if key in Lset[l]:
                break
            Lset[l][key] = len(Lset[l])
            if l > 0:
                shared[l - 1][(ids[:l - 1], key, "L")] = ids[l - 1]
        for l in range(i_sw + 1, L + 1):
            key = ids[l:]
            if key in Rset[l]:
                break
            Rset[l][key] = len(Rset[l])
            if l < L:
                shared[l][(key, ids[l + 1:], "R")] = ids[l]
        blk = switch[i_sw].setdefault((ids[:i_sw], ids[i_sw + 1:]), np.zeros((4, 4)))
        blk += coef * sign * table.mats[ids[i_sw]]
    # channel indices: left strings first (by insertion), then right strings
    R = [len(Lset[l]) + len(Rset[l]) for l in range(L + 1)]
    cores = []
    for i in range(L):
        A, Bi, O = [], [], []
        for (ka, kb, side), fid in shared[i].items():
            if side == "L":
                A.append(Lset[i][ka])
                Bi.append(Lset[i + 1][kb])
            else:
                A.append(len(Lset[i]) + Rset[i][ka])
                Bi.append(len(Lset[i + 1]) + Rset[i + 1][kb])
            O.append(table.mats[fid])
        for (ka, kb), M in switch[i].items():
            if np.any(M != 0.0):
                A.append(Lset[i][ka])
                Bi.append(len(Lset[i + 1]) + Rset[i + 1][kb])
                O.append(M)
        cores.append((np.asarray(A, dtype=np.int64), np.asarray(Bi, dtype=np.int64),
                      np.asarray(O, dtype=np.float64).reshape(-1, 4, 4)))
    assert R[0] == 1 and R[L] == 1
    return OracleMPO(L, R, cores)


def mpo_to_matrix(mpo: OracleMPO) -> np.ndarray:
    """Contract the MPO to the full 4^L x 4^L matrix (tensor-index order of
    ``oracle.fock``).  Tiny L only."""
    M = mpo.dense_core(0)[0]  # [s', s, B]
    M = M.transpose(2, 0, 1)   # [B, out, in]
    for k in range(1, mpo.L):
        W = mpo.dense_core(k)  # [A, s', s, B]
        M = np.einsum("Aoi,AstB->Bosit", M, W)
        n = M.shape[1] * 4
        M = M.reshape(M.shape[0], n, n)
    return M[0]
