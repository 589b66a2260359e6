"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module draws random numbers and lays out quantum-number (QN) structure.
It holds none of the method's arithmetic: no contraction, no orthogonalisation,
no eigensolve, no truncation.  Both sides (``oracle/`` and the HIP library)
consume exactly the same arrays produced here.

Workload recipe (stands in for the molecular integrals of the paper's
experiments, Section 4, which are not available here):

* ``h = (A + A^T)/2 + diag(linspace(-2, 0, L))`` with ``A ~ N(0, 1)``;
* ``B_k = (C_k + C_k^T)/2`` with ``C_k ~ N(0, 0.3^2)``, ``k = 1..K``;
* electron-repulsion integrals ``(pq|rs) = sum_k B_k[p,q] B_k[r,s]``
  (chemists' notation, 8-fold symmetric, positive semidefinite);
* ``numpy.random.default_rng(seed)`` draws ``A`` first, then ``C_1..C_K``.

Linear-system workload (eq. energy_lin needs a symmetric positive definite A and a
right-hand side F): A is the Hamiltonian of the same recipe with the one-body
integrals shifted by ``sigma / N`` on the diagonal, which adds ``sigma`` on the
N-electron sector.  ``sigma = 1 + N * g`` with ``g`` the Gershgorin bound
``max_p sum_q |M_pq|`` of ``M = h - 1/2 sum_k B_k B_k``: the two-electron part equals
``1/2 sum_k (sum B_k[p,q] E_pq)^2 - 1/2 sum (B_k B_k)_ps E_ps``, whose first term is
positive semidefinite, so ``H >= sum M_ps E_ps >= -N g`` and ``A >= 1`` there.  F and
the initial iterate of this workload are random QN-consistent TTs of the same sector
scaled to unit norm (``unit_tt``: the norm of a random TT grows geometrically with L).
This bound and that norm are the only arithmetic of the module beyond draws and
label structure (they define inputs).

Local basis of one spatial orbital (one tensor-train site, ``n = 4``):
``|0>, |up>, |dn>, |updn>`` with charges ``(N, 2Sz) = (0,0), (1,1), (1,-1), (2,0)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SITE_CHARGES = ((0, 0), (1, 1), (1, -1), (2, 0))
LOCAL_DIM = 4


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: problem size, truncation rank and subdomains."""

    name: str
    L: int
    n_elec: int
    two_sz: int
    n_factors: int
    seed: int
    chi: int
    lengths: tuple = field(default_factory=tuple)
    matvec_prec: str = "f64"
    dav_tol: float = 1e-8


# The five workloads: sequential DMRG (L=6), FP64 additive sweep (L=16),
# batched FP32 additive sweep (L=32), mixed-precision sweep (L=24) and the
# differentiation case (L=16).
WORKLOADS = {
    1: Workload("dmrg2_L6_chi16", 6, 6, 0, 6, 1001, 16, (), "f64", 1e-10),
    2: Workload("a2dmrg_L16_chi256_P4", 16, 16, 0, 16, 1002, 256, (4, 4, 4, 4), "f64", 1e-8),
    3: Workload("a2dmrg_L32_chi512_P8", 32, 32, 0, 32, 1003, 512, (3, 5, 4, 6, 3, 4, 3, 4), "f32", 1e-8),
    4: Workload("a2dmrg_L24_chi1024_P6", 24, 24, 0, 24, 1004, 1024, (4, 4, 4, 4, 4, 4), "bf16", 1e-8),
    5: Workload("grad_L16_chi256", 16, 16, 0, 16, 1002, 256, (), "f64", 1e-8),
}


def integrals(L: int, n_factors: int, seed: int):
    """Return ``(h, B)`` with ``h`` of shape (L, L) and ``B`` of shape (K, L, L)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((L, L))
    h = 0.5 * (A + A.T) + np.diag(np.linspace(-2.0, 0.0, L))
    B = np.empty((n_factors, L, L))
    for k in range(n_factors):
        C = rng.normal(0.0, 0.3, size=(L, L))
        B[k] = 0.5 * (C + C.T)
    return h, B


def workload_integrals(idx: int):
    w = WORKLOADS[idx]
    return integrals(w.L, w.n_factors, w.seed)


def linear_system(L: int, n_elec: int, seed: int, chi_f: int):
    """Inputs of the linear-system functional: ``(h_shift, B, sigma, F_cores,
    F_labels)``: the one-body integrals of ``integrals(L, L, seed)`` shifted so that
    A = H(h_shift, B) >= 1 on the ``n_elec``-electron sector (module docstring), and a
    random TT F of unit norm (bond dimension ``chi_f``, TT seed ``seed + 7``) of that
    sector with Sz = 0.  The initial iterate is ``unit_tt(random_mps(...))``."""
    h, B = integrals(L, L, seed)
    M = h - 0.5 * np.einsum("kpq,kqs->ps", B, B)
    g = float(np.max(np.sum(np.abs(M), axis=1)))
    sigma = 1.0 + n_elec * g
    h_shift = h + (sigma / n_elec) * np.eye(L)
    F, Fl = random_mps(L, n_elec, 0, chi_f, seed + 7)
    return h_shift, B, sigma, unit_tt(F), Fl


def unit_tt(cores):
    """The TT scaled to unit norm (last core divided by the norm, by transfer matrices)."""
    E = np.ones((1, 1))
    for U in cores:
        r, n, r2 = U.shape
        t = (E @ U.reshape(r, n * r2)).reshape(r * n, r2)   # [a s, d] = sum_b E[a, b] U[b, s, d]
        E = U.reshape(r * n, r2).T @ t                      # [c, d] = sum_{a s} U[a, s, c] t[a s, d]
    nrm = math.sqrt(float(E[0, 0]))
    out = [c.copy() for c in cores]
    out[-1] = out[-1] / nrm
    return out


# ---------------------------------------------------------------------------
# QN structure of bonds
# ---------------------------------------------------------------------------

def _count_states(nsites: int, n: int, two_sz: int) -> int:
    """Number of occupation patterns of ``nsites`` spatial orbitals with
    ``n`` electrons and spin projection ``two_sz/2``."""
    if (n + two_sz) % 2:
        return 0
    na = (n + two_sz) // 2
    nb = (n - two_sz) // 2
    if na < 0 or nb < 0 or na > nsites or nb > nsites:
        return 0
    return math.comb(nsites, na) * math.comb(nsites, nb)


def full_sector_dims(L: int, n_elec: int, two_sz: int, k: int) -> dict:
    """Exact (untruncated) sector dimensions of bond ``k`` (sites ``< k`` on the left).

    A left charge ``q`` is kept when both the left and the right part admit it;
    its dimension is ``min(#left states, #right states)``.
    """
    out = {}
    for nl in range(0, min(2 * k, n_elec) + 1):
        for szl in range(-nl, nl + 1):
            dl = _count_states(k, nl, szl)
            dr = _count_states(L - k, n_elec - nl, two_sz - szl)
            d = min(dl, dr)
            if d > 0:
                out[(nl, szl)] = d
    return out


def _apportion(full: dict, chi: int) -> dict:
    """Distribute at most ``chi`` states over sectors proportionally to ``full``
    (largest-remainder rounding, ties broken by charge order)."""
    tot = sum(full.values())
    if tot <= chi:
        return dict(full)
    keys = sorted(full)
    raw = {q: full[q] * chi / tot for q in keys}
    base = {q: min(full[q], int(math.floor(raw[q]))) for q in keys}
    left = chi - sum(base.values())
    order = sorted(keys, key=lambda q: (-(raw[q] - math.floor(raw[q])), q))
    for q in order:
        if left <= 0:
            break
        if base[q] < full[q]:
            base[q] += 1
            left -= 1
    return {q: d for q, d in base.items() if d > 0}


def bond_sectors(L: int, n_elec: int, two_sz: int, chi: int):
    """Sector dimensions for every bond ``0..L`` of a chi-bounded QN-consistent TT.

    Returns a list of dicts ``{charge: dim}``.  Each dimension is made
    compatible with both neighbours (a sector cannot be larger than what the
    adjacent bond and one site can feed), so random cores built on this
    structure have full rank in every block.
    """
    dims = [_apportion(full_sector_dims(L, n_elec, two_sz, k), chi) for k in range(L + 1)]
    dims[0] = {(0, 0): 1}
    dims[L] = {(n_elec, two_sz): 1}
    for _ in range(2):
        for k in range(1, L + 1):
            for q in list(dims[k]):
                feed = sum(dims[k - 1].get((q[0] - c[0], q[1] - c[1]), 0) for c in SITE_CHARGES)
                dims[k][q] = min(dims[k][q], feed)
                if dims[k][q] == 0:
                    del dims[k][q]
        for k in range(L - 1, -1, -1):
            for q in list(dims[k]):
                feed = sum(dims[k + 1].get((q[0] + c[0], q[1] + c[1]), 0) for c in SITE_CHARGES)
                dims[k][q] = min(dims[k][q], feed)
                if dims[k][q] == 0:
                    del dims[k][q]
    return dims


def bond_labels(sectors: dict) -> np.ndarray:
    """Expand ``{charge: dim}`` into an ``(r, 2)`` int32 label array sorted by charge."""
    rows = []
    for q in sorted(sectors):
        rows.extend([q] * sectors[q])
    return np.asarray(rows, dtype=np.int32).reshape(-1, 2)


def allowed_mask(ql: np.ndarray, qr: np.ndarray) -> np.ndarray:
    """Boolean mask ``[a, s, b]`` of QN-allowed entries of a core with left
    labels ``ql`` and right labels ``qr`` (``q(a) + q(s) == q(b)``).  Pure
    structure: used to place random numbers."""
    sc = np.asarray(SITE_CHARGES, dtype=np.int32)
    tot = ql[:, None, None, :] + sc[None, :, None, :]
    return np.all(tot == qr[None, None, :, :], axis=-1)


def random_mps(L: int, n_elec: int, two_sz: int, chi: int, seed: int):
    """Random QN-consistent TT: cores ``U[k]`` of shape ``(r_k, 4, r_{k+1})`` and
    bond labels ``q[k]`` of shape ``(r_k, 2)``.  Entries are ``N(0,1)`` on the
    allowed blocks and zero elsewhere.  The cores are NOT orthogonalised."""
    rng = np.random.default_rng(seed)
    secs = bond_sectors(L, n_elec, two_sz, chi)
    labels = [bond_labels(s) for s in secs]
    cores = []
    for k in range(L):
        m = allowed_mask(labels[k], labels[k + 1])
        U = np.zeros(m.shape)
        U[m] = rng.standard_normal(int(m.sum()))
        cores.append(U)
    return cores, labels


def random_dense(shape, seed: int, scale: float = 1.0):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(shape)


def random_sparse_mpo_core(R_left: int, R_right: int, nnz_per_col: int, seed: int):
    """Random sparse MPO core for kernel-level tests: ``nnz`` entries
    ``(A, B, op[4][4])``.  Every right channel ``B`` receives ``nnz_per_col``
    entries from distinct left channels; local operators are dense N(0,1)."""
    rng = np.random.default_rng(seed)
    A_idx, B_idx = [], []
    for b in range(R_right):
        k = min(nnz_per_col, R_left)
        A_idx.extend(rng.choice(R_left, size=k, replace=False).tolist())
        B_idx.extend([b] * k)
    A_idx = np.asarray(A_idx, dtype=np.int32)
    B_idx = np.asarray(B_idx, dtype=np.int32)
    ops = rng.standard_normal((len(A_idx), LOCAL_DIM, LOCAL_DIM))
    return A_idx, B_idx, ops


def heff_operands(rl: int, rr: int, R_l: int, R_m: int, R_r: int, seed: int, nnz_per_col: int = 3):
    """Random operands of one two-site effective-Hamiltonian product:
    left env ``L[A][a'][a]``, right env ``R[C][b'][b]``, two sparse MPO cores
    and a two-site tensor ``x[a][s1][s2][b]``."""
    rng = np.random.default_rng(seed)
    Lenv = rng.standard_normal((R_l, rl, rl)) / math.sqrt(rl)
    Renv = rng.standard_normal((R_r, rr, rr)) / math.sqrt(rr)
    x = rng.standard_normal((rl, LOCAL_DIM, LOCAL_DIM, rr))
    s1, s2 = rng.integers(0, 2**31 - 1, size=2)
    W1 = random_sparse_mpo_core(R_l, R_m, nnz_per_col, int(s1))
    W2 = random_sparse_mpo_core(R_m, R_r, nnz_per_col, int(s2))
    return Lenv, W1, W2, Renv, x
