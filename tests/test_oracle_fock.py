"""Pins of the Fock-space Hamiltonian and exact diagonalisation (Section 3.2)."""
import itertools

import numpy as np
import pytest

import seeded_inputs as S
from oracle import fock as F


@pytest.mark.parametrize("L", [2, 3])
def test_factorised_hamiltonian_equals_term_by_term_definition(L):
    h, B = S.integrals(L, L, 7 + L)
    eri = np.einsum("kpq,krs->pqrs", B, B)
    Hd = F.hamiltonian_direct(h, eri)
    Hf = F.hamiltonian(h, B, F.all_states(L))
    assert np.abs(Hd - Hf).max() < 1e-12
    assert np.abs(Hd - Hd.T).max() < 1e-13


def test_hubbard_dimer_closed_form():
    # two sites, hopping t, on-site repulsion U: E0 = (U - sqrt(U^2 + 16 t^2))/2
    for t, U in [(1.0, 3.0), (0.7, 0.5), (1.3, 8.0)]:
        h = np.array([[0.0, -t], [-t, 0.0]])
        B = np.zeros((2, 2, 2))
        B[0, 0, 0] = np.sqrt(U)
        B[1, 1, 1] = np.sqrt(U)
        E, _, _ = F.ed_ground(h, B, 2, 0)
        assert abs(E - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-12


def test_one_body_closed_shell_energy():
    # without two-body terms the ground state fills the lowest orbitals twice
    h, _ = S.integrals(5, 1, 11)
    B = np.zeros((1, 5, 5))
    eps = np.linalg.eigvalsh(h)
    for n in (2, 4, 6):
        E, _, _ = F.ed_ground(h, B, n, 0)
        assert abs(E - 2 * eps[: n // 2].sum()) < 1e-11


def test_single_orbital_double_occupancy():
    h = np.array([[-0.8]])
    B = np.array([[[1.1]], [[0.4]]])
    U = 1.1**2 + 0.4**2
    E, _, _ = F.ed_ground(h, B, 2, 0)
    assert abs(E - (2 * -0.8 + U)) < 1e-13


def test_sector_dimension_and_quantum_numbers():
    L = 6
    st = F.sector_states(L, 6, 0)
    assert len(st) == 400
    N, Sz2 = F.number_ops(st, L)
    assert np.all(N == 6) and np.all(Sz2 == 0)
    # H is closed on the sector: building it on the full space and restricting agrees
    h, B = S.integrals(4, 4, 3)
    full = F.all_states(4)
    Hfull = F.hamiltonian(h, B, full)
    sec = F.sector_states(4, 4, 0)
    idx = F.tensor_index(sec, 4)
    Hsec = F.hamiltonian(h, B, sec)
    assert np.abs(Hfull[np.ix_(idx, idx)] - Hsec).max() < 1e-12
    other = np.setdiff1d(np.arange(len(full)), idx)
    assert np.abs(Hfull[np.ix_(other, idx)]).max() < 1e-12


def test_one_rdm_properties_and_linearity():
    h, B = S.workload_integrals(1)
    E0, psi, st = F.ed_ground(h, B, 6, 0)
    g = F.one_rdm(psi, st, 6)
    assert abs(np.trace(g) - 6) < 1e-10
    assert np.abs(g - g.T).max() < 1e-12
    w = np.linalg.eigvalsh(g)
    assert w.min() > -1e-10 and w.max() < 2 + 1e-10
    # E(h) = <psi|H(h)|psi> is linear in h: central differences are exact
    Hs = F.hamiltonian(h, B, st)
    for p, q in [(0, 0), (1, 3), (4, 2)]:
        d = 1e-5
        hp = h.copy(); hp[p, q] += d
        hm = h.copy(); hm[p, q] -= d
        Ep = psi @ F.hamiltonian(hp, B, st) @ psi
        Em = psi @ F.hamiltonian(hm, B, st) @ psi
        assert abs((Ep - Em) / (2 * d) - g[p, q]) < 1e-8
    assert abs(psi @ Hs @ psi - E0) < 1e-10
