"""Pins of the transfer-matrix one-particle density matrix (oracle.density)
against the dense Fock-space definition (oracle.fock), and against closed
forms (occupation-number states)."""
import numpy as np

import seeded_inputs as S
from oracle import density as D
from oracle import fock as F
from oracle import tt as T


def test_matches_dense_definition_random_tt():
    # random TT without charge structure on all 4^L states: every sign of the
    # Jordan-Wigner strings enters
    rng = np.random.default_rng(5)
    L, r = 4, [1, 3, 5, 3, 1]
    cores = [rng.standard_normal((r[k], 4, r[k + 1])) for k in range(L)]
    psi = T.contract_full(cores)
    psi /= np.linalg.norm(psi)
    st = F.all_states(L)
    g_dense = F.one_rdm(psi, st, L)
    g_tt = D.one_rdm(cores)
    assert np.abs(g_tt - g_dense).max() < 1e-12


def test_matches_dense_definition_qn_tt():
    L = 6
    cores, labels = S.random_mps(L, L, 0, 16, 77)
    psi = T.contract_full(cores)
    st = F.sector_states(L, L, 0)
    y = psi[F.tensor_index(st, L)]
    assert abs(np.linalg.norm(y) - np.linalg.norm(psi)) < 1e-12  # the state lies in the sector
    y /= np.linalg.norm(y)
    g = D.one_rdm(cores)
    assert np.abs(g - F.one_rdm(y, st, L)).max() < 1e-12
    assert abs(np.trace(g) - L) < 1e-12


def test_occupation_state_closed_form():
    # product state with local states i_p: gamma = diag(n_p), no off-diagonal
    loc = [3, 1, 0, 2, 3, 0]
    cores = []
    for i in loc:
        U = np.zeros((1, 4, 1))
        U[0, i, 0] = 1.0
        cores.append(U)
    g = D.one_rdm(cores)
    n = np.array([bin(i).count("1") for i in loc], dtype=float)
    assert np.array_equal(g, np.diag(n))
