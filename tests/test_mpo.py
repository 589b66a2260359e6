"""The host-side MPO builder against the oracle's Fock-space Hamiltonian."""
import json
import os

import numpy as np
import pytest

import seeded_inputs as S
from oracle import fock as F
from oracle import tt as T
from paper_2505_23429_amd.mpo import build_mpo, mpo_to_matrix


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_mpo_contracts_to_hamiltonian(L):
    h, B = S.integrals(L, L, 100 + L)
    mpo = build_mpo(h, B)
    H = F.hamiltonian(h, B, F.all_states(L))
    assert np.abs(mpo_to_matrix(mpo) - H).max() < 1e-12


@pytest.mark.parametrize("switch", [1, 2, 3])
def test_mpo_switch_position_does_not_change_operator(switch):
    h, B = S.integrals(4, 3, 77)
    H = F.hamiltonian(h, B, F.all_states(4))
    assert np.abs(mpo_to_matrix(build_mpo(h, B, switch=switch)) - H).max() < 1e-12


@pytest.mark.parametrize("L", [8, 16, 24])
def test_mpo_bond_dimension(L):
    h, B = S.integrals(L, L, 5)
    mpo = build_mpo(h, B)
    assert mpo.R[0] == 1 and mpo.R[L] == 1
    assert mpo.R[L // 2] == 2 * L * L + 3 * L + 2
    assert max(mpo.R) == mpo.R[L // 2]


def test_mpo_channel_charges_are_conserved():
    # every entry W[A,s',s,B] is non-zero only if q(A) + q(s') = q(B) + q(s)
    h, B = S.integrals(6, 6, 9)
    mpo = build_mpo(h, B)
    sq = np.array(S.SITE_CHARGES)
    for k in range(6):
        for a, b, op in zip(mpo.A[k], mpo.B[k], mpo.ops[k]):
            nz = np.argwhere(np.abs(op) > 0)
            for sp, s in nz:
                lhs = mpo.chan_q[k][a] + sq[sp] - sq[s]
                assert np.all(lhs == mpo.chan_q[k + 1][b])


def test_mpo_energy_expectation_at_L8():
    # <psi|H|psi> of a random TT: MPO environment chain vs the sector Hamiltonian
    from oracle import contract as C
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ed_energies.json")))
    h, B = S.integrals(8, 8, 1008)
    mpo = build_mpo(h, B)
    prob = T.Problem(h, B, 8, 0)
    cores, labels = S.random_mps(8, 8, 0, 12, 55)
    cores = T.left_orthogonalize(cores, labels)
    E = np.ones((1, 1, 1))
    for k in range(8):
        E = C.env_left(E, cores[k], mpo.dense_core(k), cores[k])
    nrm = np.sum(T.contract_full(cores) ** 2)
    assert abs(E[0, 0, 0] / nrm - prob.energy(cores)) < 1e-10
    assert prob.energy(cores) >= golden["ed_L8_N8_seed1008"]["E0"] - 1e-12
