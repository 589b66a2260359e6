"""One-particle density matrix of a tensor-train state without a dense vector.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

``gamma_pq = <Psi|E_pq|Psi> / <Psi|Psi>`` with ``E_pq = sum_s a^+_{ps} a_{qs}``
(the one-body part of the Hamiltonian of Section 3.2).  Because the energy
``<Psi|H(h)|Psi>`` of a fixed state is linear in the one-body integrals,
``dE/dh_pq = gamma_pq``.

The operator ``a^+_{ps} a_{qs}`` is written as a product of 4x4 site factors
in the Jordan-Wigner convention of ``oracle.fock`` (spin orbitals ordered
``(0a, 0b, 1a, 1b, ...)``, ``a^+_j |n> = (-1)^{sum_{i<j} n_i} |n + e_j>``,
local basis ``|0>, |up>, |dn>, |updn>`` with index ``n_a + 2 n_b``), and its
expectation value is one left-to-right transfer-matrix contraction through
the cores (Definition "tensor train contraction mapping"): cost
``O(L n r^3)`` per entry, so it reaches the L = 16, chi = 256 states that the
dense sector vector of ``oracle.fock`` cannot hold.
"""
from __future__ import annotations

import numpy as np

# site factors (row = output state, column = input state)
_P = np.diag([1.0, -1.0, -1.0, 1.0])          # parity (-1)^(n_a + n_b)
_CDAG = {
    0: np.array([[0, 0, 0, 0], [1, 0, 0, 0], [0, 0, 0, 0], [0, 0, 1, 0]], dtype=float),   # alpha: no sign inside the site
    1: np.array([[0, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 0], [0, -1, 0, 0]], dtype=float),  # beta: sign (-1)^(n_a)
}
_I = np.eye(4)


def hopping_factors(L: int, p: int, q: int, s: int):
    """Site factors of a^+_{ps} a_{qs}: the product of the two operators' Jordan-
    Wigner strings and local factors, site by site."""
    cdag = _CDAG[s]
    c = cdag.T
    ops = []
    for i in range(L):
        A = _P if i < p else (cdag if i == p else _I)   # a^+_{ps}
        B = _P if i < q else (c if i == q else _I)      # a_{qs}
        ops.append(A @ B)
    return ops


def expectation(cores, ops) -> float:
    """<Psi|prod_i O_i|Psi> / <Psi|Psi> by transfer matrices (real cores U[a][s][b])."""
    E = np.ones((1, 1))
    N = np.ones((1, 1))
    for U, O in zip(cores, ops):
        # E'[b', b] = sum E[a', a] U[a', s', b'] O[s', s] U[a, s, b]
        T = np.einsum("xa,asb->xsb", E, U, optimize=True)
        T = np.einsum("ts,xsb->xtb", O, T, optimize=True)
        E = np.einsum("xtc,xtb->cb", U, T, optimize=True)
        M = np.einsum("xa,asb->xsb", N, U, optimize=True)
        N = np.einsum("xsc,xsb->cb", U, M, optimize=True)
    return float(E[0, 0] / N[0, 0])


def one_rdm_entry(cores, p: int, q: int) -> float:
    L = len(cores)
    return sum(expectation(cores, hopping_factors(L, p, q, s)) for s in (0, 1))


def one_rdm(cores) -> np.ndarray:
    L = len(cores)
    return np.array([[one_rdm_entry(cores, p, q) for q in range(L)] for p in range(L)])
