"""Second-quantised electronic Hamiltonian on the Fock space (Section 3.2).

Spin orbitals are ordered ``(0a, 0b, 1a, 1b, ...)``; an occupation pattern is
an integer whose bit ``2p + s`` is the occupation of spatial orbital ``p`` with
spin ``s`` (0 = alpha, 1 = beta).  Creation/annihilation follow the
Jordan-Wigner convention: ``a^+_j |n> = (-1)^{sum_{i<j} n_i} |n + e_j>``.

The tensor index of a basis state (the isomorphism of the Fock space with
the tensor space) is ``sum_p i_p 4^(L-1-p)`` with the local index
``i_p = n_{p,alpha} + 2 n_{p,beta}``, i.e. the local basis
``|0>, |up>, |dn>, |updn>``.

Hamiltonian (chemists' notation for the two-electron integrals):

    H = sum_{pq} h_pq sum_s a^+_{ps} a_{qs}
      + 1/2 sum_{pqrs} (pq|rs) sum_{s,t} a^+_{ps} a^+_{rt} a_{st} a_{qs}

With ``(pq|rs) = sum_k B_k[p,q] B_k[r,s]`` the operator identity
``sum (pq|rs) a^+ a^+ a a = sum_k O_k^2 - sum_ps (sum_k B_k^2)_ps E_ps``,
``O_k = sum_pq B_k[p,q] E_pq`` and ``E_pq = sum_s a^+_{ps} a_{qs}``, gives the
sector matrix from one-body excitation matrices only.  ``hamiltonian_direct``
builds the same operator term by term from the definition for tiny ``L``; the
tests pin the two against each other.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def _popcount(x):
    return np.bitwise_count(np.asarray(x, dtype=np.uint64)).astype(np.int64)


def sector_states(L: int, n_elec: int, two_sz: int) -> np.ndarray:
    """Occupation patterns (uint64) with ``n_elec`` electrons and spin ``two_sz/2``,
    sorted by tensor index."""
    na = (n_elec + two_sz) // 2
    nb = (n_elec - two_sz) // 2
    out = []
    for ca in itertools.combinations(range(L), na):
        for cb in itertools.combinations(range(L), nb):
            s = 0
            for p in ca:
                s |= 1 << (2 * p)
            for p in cb:
                s |= 1 << (2 * p + 1)
            out.append(s)
    out = np.asarray(out, dtype=np.uint64)
    idx = tensor_index(out, L)
    return out[np.argsort(idx)]


def tensor_index(states: np.ndarray, L: int) -> np.ndarray:
    """Flat tensor index of occupation patterns (local index ``n_a + 2 n_b``)."""
    states = np.asarray(states, dtype=np.uint64)
    idx = np.zeros(states.shape, dtype=np.int64)
    for p in range(L):
        na = ((states >> np.uint64(2 * p)) & np.uint64(1)).astype(np.int64)
        nb = ((states >> np.uint64(2 * p + 1)) & np.uint64(1)).astype(np.int64)
        idx = idx * 4 + na + 2 * nb
    return idx


def all_states(L: int) -> np.ndarray:
    """All 4^L occupation patterns, ordered by tensor index."""
    idx = np.arange(4**L, dtype=np.int64)
    st = np.zeros(idx.shape, dtype=np.uint64)
    rem = idx.copy()
    for p in range(L - 1, -1, -1):
        loc = rem % 4
        rem //= 4
        na = (loc & 1).astype(np.uint64)
        nb = ((loc >> 1) & 1).astype(np.uint64)
        st |= na << np.uint64(2 * p)
        st |= nb << np.uint64(2 * p + 1)
    return st


def _apply_op(states, so, create):
    """Apply a^+_so (create=True) or a_so to every pattern. Returns (new, sign, ok)."""
    bit = np.uint64(1) << np.uint64(so)
    occ = (states & bit) != 0
    ok = ~occ if create else occ
    below = _popcount(states & (bit - np.uint64(1)))
    sign = np.where(below % 2 == 0, 1.0, -1.0)
    new = states ^ bit
    return new, sign, ok


def excitation(states: np.ndarray, p: int, q: int, spin: int, index_of) -> sp.csr_matrix:
    """Matrix of ``a^+_{p,spin} a_{q,spin}`` on the basis ``states``."""
    s1, sg1, ok1 = _apply_op(states, 2 * q + spin, create=False)
    s2, sg2, ok2 = _apply_op(s1, 2 * p + spin, create=True)
    ok = ok1 & ok2
    cols = np.nonzero(ok)[0]
    rows = index_of(s2[ok])
    vals = (sg1 * sg2)[ok]
    D = len(states)
    return sp.csr_matrix((vals, (rows, cols)), shape=(D, D))


def _indexer(states):
    order = np.argsort(states)
    sorted_states = states[order]

    def index_of(s):
        pos = np.searchsorted(sorted_states, s)
        if np.any(pos >= len(states)) or np.any(sorted_states[np.minimum(pos, len(states) - 1)] != s):
            raise ValueError("state left the basis")
        return order[pos]

    return index_of


def one_body_matrices(states: np.ndarray, L: int):
    """``E[p][q] = sum_s a^+_{ps} a_{qs}`` as sparse matrices on ``states``."""
    index_of = _indexer(states)
    E = [[None] * L for _ in range(L)]
    for p in range(L):
        for q in range(L):
            E[p][q] = excitation(states, p, q, 0, index_of) + excitation(states, p, q, 1, index_of)
    return E


def hamiltonian(h: np.ndarray, B: np.ndarray, states: np.ndarray, dense: bool = True):
    """Hamiltonian restricted to the basis ``states`` (must be closed under H)."""
    L = h.shape[0]
    E = one_body_matrices(states, L)
    D = len(states)
    htil = h - 0.5 * np.einsum("kpq,kqs->ps", B, B)
    H = sp.csr_matrix((D, D))
    for p in range(L):
        for q in range(L):
            if htil[p, q] != 0.0:
                H = H + htil[p, q] * E[p][q]
    for k in range(B.shape[0]):
        O = sp.csr_matrix((D, D))
        for p in range(L):
            for q in range(L):
                if B[k, p, q] != 0.0:
                    O = O + B[k, p, q] * E[p][q]
        H = H + 0.5 * (O @ O)
    return H.toarray() if dense else H.tocsr()


def hamiltonian_direct(h: np.ndarray, eri: np.ndarray) -> np.ndarray:
    """Term-by-term Hamiltonian on the full Fock space (tensor-index order) for
    tiny ``L``; ``eri[p,q,r,s] = (pq|rs)``.  Pure-Python loops, definition only."""
    L = h.shape[0]
    st = all_states(L)
    D = len(st)
    pos = {int(s): i for i, s in enumerate(st)}

    def apply(ops, s):
        sign = 1.0
        for so, create in reversed(ops):
            bit = 1 << so
            occ = bool(s & bit)
            if occ == create:
                return None, 0.0
            if bin(s & (bit - 1)).count("1") % 2:
                sign = -sign
            s ^= bit
        return s, sign

    H = np.zeros((D, D))
    for j, s in enumerate(st):
        s = int(s)
        for p in range(L):
            for q in range(L):
                for a in range(2):
                    t, sg = apply([(2 * p + a, True), (2 * q + a, False)], s)
                    if t is not None:
                        H[pos[t], j] += h[p, q] * sg
        for p, q, r, u in itertools.product(range(L), repeat=4):
            v = eri[p, q, r, u]
            if v == 0.0:
                continue
            for a in range(2):
                for b in range(2):
                    ops = [(2 * p + a, True), (2 * r + b, True), (2 * u + b, False), (2 * q + a, False)]
                    t, sg = apply(ops, s)
                    if t is not None:
                        H[pos[t], j] += 0.5 * v * sg
    return H


def ed_ground(h: np.ndarray, B: np.ndarray, n_elec: int, two_sz: int = 0):
    """Lowest eigenpair of H in the (N, Sz) sector.  Returns ``(E0, psi, states)``
    with ``psi`` indexed like ``states``."""
    L = h.shape[0]
    st = sector_states(L, n_elec, two_sz)
    H = hamiltonian(h, B, st, dense=True)
    w, v = np.linalg.eigh(H)
    return w[0], v[:, 0], st


def embed(psi_sector: np.ndarray, states: np.ndarray, L: int) -> np.ndarray:
    """Scatter a sector vector into the full 4^L tensor (flattened)."""
    full = np.zeros(4**L)
    full[tensor_index(states, L)] = psi_sector
    return full


def restrict(psi_full: np.ndarray, states: np.ndarray, L: int) -> np.ndarray:
    return psi_full[tensor_index(states, L)]


def one_rdm(psi_sector: np.ndarray, states: np.ndarray, L: int) -> np.ndarray:
    """Spin-summed one-particle density matrix ``gamma_pq = <psi|E_pq|psi>``
    (for a normalised real ``psi``)."""
    E = one_body_matrices(states, L)
    g = np.empty((L, L))
    for p in range(L):
        for q in range(L):
            g[p, q] = psi_sector @ (E[p][q] @ psi_sector)
    return g


def number_ops(states: np.ndarray, L: int):
    """Diagonals of the particle-number and ``2 Sz`` operators on ``states``."""
    st = np.asarray(states, dtype=np.uint64)
    na = np.zeros(len(st), dtype=np.int64)
    nb = np.zeros(len(st), dtype=np.int64)
    for p in range(L):
        na += ((st >> np.uint64(2 * p)) & np.uint64(1)).astype(np.int64)
        nb += ((st >> np.uint64(2 * p + 1)) & np.uint64(1)).astype(np.int64)
    return na + nb, na - nb
