"""Whole-path parity: the HIP library's two-site DMRG and additive two-level
sweeps against the oracle from identical inputs (|dE| <= 1e-8 Ha in FP64,
<= 1e-6 Ha with FP32/BF16 products and FP64 refinement)."""
import json
import os

import numpy as np
import pytest

import seeded_inputs as S
from oracle import fock as F
from oracle import tt as T

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ed_energies.json")))


def _setup(L, seed_int, chi, seed_mps, chi0=None):
    from paper_2505_23429_amd.mpo import build_mpo

    h, B = S.integrals(L, L, seed_int)
    mpo = build_mpo(h, B)
    cores, labels = S.random_mps(L, L, 0, chi0 or chi, seed_mps)
    prob = T.Problem(h, B, L, 0)
    oc = T.left_orthogonalize(cores, labels)
    return mpo, cores, labels, prob, oc


def _gauge(S_, A_, c):
    """Signs d_j with d_j * S[0, j] >= 0 (each subdomain update is an eigenvector,
    defined up to sign), then the overall sign of c that makes its largest entry
    positive, so that c is compared with its signs."""
    d = np.sign(S_[0])
    d[0] = 1.0
    d[d == 0] = 1.0
    Sg, Ag, cg = S_ * np.outer(d, d), A_ * np.outer(d, d), c * d
    i = int(np.argmax(np.abs(cg)))
    return Sg, Ag, (-cg if cg[i] < 0 else cg)


def _ctx(mpo, cores, labels, **kw):
    from paper_2505_23429_amd.api import open_context

    return open_context(mpo, cores, labels, **kw)


def test_energy_of_initial_state_L8():
    mpo, cores, labels, prob, oc = _setup(8, 1008, 24, 7)
    ctx = _ctx(mpo, cores, labels, chi=24)
    assert abs(ctx.energy() - prob.energy(oc)) < 1e-10
    # the device left-orthogonalisation reproduces the same state
    c2, l2 = ctx.get_mps()
    assert abs(prob.energy(c2) - prob.energy(oc)) < 1e-10
    for U in c2[:-1]:
        M = U.reshape(-1, U.shape[2])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() < 1e-12


def test_dmrg2_full_rank_equals_ed():
    mpo, cores, labels, prob, oc = _setup(6, 1001, 64, 2001)
    ctx = _ctx(mpo, cores, labels, chi=64, dav_tol=1e-10)
    E, rc = ctx.dmrg2(1)
    assert abs(E[-1] - GOLD["ed_L6_N6_seed1001"]["E0"]) < 1e-10


def test_dmrg2_truncated_matches_oracle():
    mpo, cores, labels, prob, oc = _setup(6, 1001, 16, 2002)
    ctx = _ctx(mpo, cores, labels, chi=16, dav_tol=1e-10)
    E, rc = ctx.dmrg2(2)
    Eo, _, _ = T.dmrg2(prob, oc, labels, 16, nsweeps=2)
    assert np.abs(np.array(E) - np.array(Eo)).max() < 1e-8


@pytest.mark.parametrize("L,seed,chi,lengths", [(6, 1001, 16, (2, 2, 2)), (8, 1008, 16, (3, 3, 2)),
                                                 (8, 1008, 24, (2, 3, 3))])
def test_a2dmrg_sweep_matches_oracle(L, seed, chi, lengths):
    mpo, cores, labels, prob, oc = _setup(L, seed, chi, 3 + chi)
    ctx = _ctx(mpo, cores, labels, chi=chi, dav_tol=1e-10)
    rep = ctx.sweep(list(lengths))
    ro = T.a2dmrg_sweep(prob, oc, labels, chi, lengths)
    assert abs(rep["E_before"] - prob.energy(oc)) < 1e-10
    assert np.abs(rep["E_local"] - np.array(ro.E_local)).max() < 1e-8
    # each local eigenvector is defined up to sign: compare in the gauge S[0, j] >= 0
    Sg, Ag, cg = _gauge(rep["S"], rep["A"], rep["c"])
    So, Ao, co = _gauge(ro.S, ro.A, ro.c)
    assert np.abs(Sg - So).max() < 1e-8
    assert np.abs(Ag - Ao).max() < 1e-8
    assert np.abs(cg - co).max() < 1e-7
    assert abs(rep["lambda"] - ro.lam) < 1e-8
    assert abs(rep["E_after"] - ro.E_new) < 1e-8
    # invariants of the coarse problem
    assert rep["lambda"] <= rep["A"][0, 0] + 1e-12
    # the iterate handed back is left-orthogonal and has the oracle energy
    c2, l2 = ctx.get_mps()
    assert abs(prob.energy(c2) - ro.E_new) < 1e-8
    assert max(q.shape[0] for q in l2) <= chi


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_a2dmrg_sweep_product_forms_match_oracle(form, prec):
    """The sweep with the other two forms of the two-site product (only the left
    operator precontracted, or none) against the dense-vector oracle, in FP64 and with
    FP32 products and the FP64 refinement."""
    L, seed, chi, lengths = 8, 1008, 24, (2, 3, 3)
    mpo, cores, labels, prob, oc = _setup(L, seed, chi, 3 + chi)
    kw = dict(matvec_prec=prec, refine_fp64=True) if prec == "f32" else {}
    ctx = _ctx(mpo, cores, labels, chi=chi, dav_tol=1e-10, precontract=form, **kw)
    rep = ctx.sweep(list(lengths))
    ro = T.a2dmrg_sweep(prob, oc, labels, chi, lengths)
    tol = 1e-8 if prec == "f64" else 1e-6
    assert np.abs(rep["E_local"] - np.array(ro.E_local)).max() < tol
    assert abs(rep["lambda"] - ro.lam) < tol
    assert abs(rep["E_after"] - ro.E_new) < tol
    c2, _ = ctx.get_mps()
    assert abs(prob.energy(c2) - ro.E_new) < tol


def test_a2dmrg_sweep_global_memory_svd_matches_oracle():
    """The same sweep with every sector SVD block factored by the global-memory path of
    the Jacobi kernel (at these sizes the blocks would otherwise all fit in LDS)."""
    L, seed, chi, lengths = 8, 1008, 24, (2, 3, 3)
    mpo, cores, labels, prob, oc = _setup(L, seed, chi, 3 + chi)
    ctx = _ctx(mpo, cores, labels, chi=chi, dav_tol=1e-10, svd_lds=False)
    rep = ctx.sweep(list(lengths))
    ro = T.a2dmrg_sweep(prob, oc, labels, chi, lengths)
    assert np.abs(rep["E_local"] - np.array(ro.E_local)).max() < 1e-8
    assert abs(rep["lambda"] - ro.lam) < 1e-8
    assert abs(rep["E_after"] - ro.E_new) < 1e-8
    c2, _ = ctx.get_mps()
    assert abs(prob.energy(c2) - ro.E_new) < 1e-8
    for U in c2[:-1]:
        M = U.reshape(-1, U.shape[2])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() < 1e-12


def test_a2dmrg_full_rank_single_sweep_exact():
    mpo, cores, labels, prob, oc = _setup(6, 1001, 64, 2001)
    ctx = _ctx(mpo, cores, labels, chi=64, dav_tol=1e-10)
    rep = ctx.sweep([2, 2, 2])
    assert abs(rep["E_after"] - GOLD["ed_L6_N6_seed1001"]["E0"]) < 1e-10


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_a2dmrg_mixed_precision_with_refinement(prec):
    L, chi, lengths = 8, 16, (3, 3, 2)
    mpo, cores, labels, prob, oc = _setup(L, 1008, chi, 19)
    ctx = _ctx(mpo, cores, labels, chi=chi, dav_tol=1e-9, matvec_prec=prec, refine_fp64=True, lowprec_tol=1e-4)
    rep = ctx.sweep(list(lengths))
    ro = T.a2dmrg_sweep(prob, oc, labels, chi, lengths)
    assert abs(rep["E_after"] - ro.E_new) < 1e-6
    assert abs(rep["lambda"] - ro.lam) < 1e-6


def test_energy_gradient_is_one_rdm():
    from paper_2505_23429_amd.mpo import h_gradient

    mpo, cores, labels, prob, oc = _setup(6, 1001, 16, 41)
    ctx = _ctx(mpo, cores, labels, chi=16)
    E, gops = ctx.mpo_gradient(mpo)
    g = h_gradient(mpo, gops)
    y = prob.to_sector(T.contract_full(oc))
    y /= np.linalg.norm(y)
    gamma = F.one_rdm(y, prob.states, 6)
    assert abs(E - prob.energy(oc)) < 1e-10
    assert np.abs(g - gamma).max() < 1e-9
    assert abs(np.trace(g) - 6) < 1e-9


def test_block_sparse_sweep_matches_dense():
    """The quantum-number block-sparse product (default) and the dense product
    give the same converged sweep (bond dimensions above one GEMM tile, stage-4
    K split, coefficient-block windows).  Unconverged local solves are not
    compared: rounding differences of two correct products grow through the
    truncations of a sweep whose eigenvectors are not yet determined."""
    from paper_2505_23429_amd.mpo import build_mpo

    L, chi, lengths = 12, 160, [4, 4, 4]
    h, B = S.integrals(L, L, 1012)
    mpo = build_mpo(h, B)
    cores, labels = S.random_mps(L, L, 0, chi, 23)
    reps = []
    for skip in (False, True):
        ctx = _ctx(mpo, cores, labels, chi=chi, dav_tol=1e-10, dav_maxiter=600, qn_skip=skip)
        reps.append(ctx.sweep(lengths))
        assert reps[-1]["status"] != 1  # TT_WNOCONV: a local solve stopped unconverged
        ctx.close()
    a, b = reps
    assert np.abs(a["E_local"] - b["E_local"]).max() < 1e-8
    assert abs(a["lambda"] - b["lambda"]) < 1e-8
    assert abs(a["E_after"] - b["E_after"]) < 1e-8


@pytest.mark.timeout(600)
@pytest.mark.parametrize("L,chi,seed", [(12, 160, 1012), (32, 512, 1003)])
def test_block_sparse_environments_match_dense(L, chi, seed):
    """<U|H|U> through the chain of block-sparse environment updates (default)
    and through the dense updates, on a chi-saturated random iterate."""
    from paper_2505_23429_amd.mpo import build_mpo

    h, B = S.integrals(L, L, seed)
    mpo = build_mpo(h, B)
    cores, labels = S.random_mps(L, L, 0, chi, seed + 1)
    E = []
    for skip in (True, False):
        ctx = _ctx(mpo, cores, labels, chi=chi, qn_skip=skip)
        E.append(ctx.energy())
        ctx.close()
    assert abs(E[0] - E[1]) < 1e-11 * max(1.0, abs(E[1]))


@pytest.mark.parametrize("mode", [2, 3, 4])
def test_a2dmrg_sweep_blocked_svd_matches_oracle(mode):
    """The same sweep with every sector SVD block of two or more columns factored by the
    blocked Jacobi kernels, whose column pairs are spread over many workgroups, with each
    variant of their pair kernels (4 rows per lane in registers as chosen by size, loops
    over LDS, 9 rows per lane): the sweep agrees with the oracle and the cores are
    isometries."""
    L, seed, chi, lengths = 8, 1008, 24, (2, 3, 3)
    mpo, cores, labels, prob, oc = _setup(L, seed, chi, 3 + chi)
    print(f"svd_blocked={mode}", flush=True)
    ctx = _ctx(mpo, cores, labels, chi=chi, dav_tol=1e-10, svd_blocked=mode)
    rep = ctx.sweep(list(lengths))
    ro = T.a2dmrg_sweep(prob, oc, labels, chi, lengths)
    assert np.abs(rep["E_local"] - np.array(ro.E_local)).max() < 1e-8
    assert abs(rep["lambda"] - ro.lam) < 1e-8
    assert abs(rep["E_after"] - ro.E_new) < 1e-8
    c2, _ = ctx.get_mps()
    assert abs(prob.energy(c2) - ro.E_new) < 1e-8
    for U in c2[:-1]:
        M = U.reshape(-1, U.shape[2])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() < 1e-12


@pytest.mark.timeout(600)
def test_full_size_sweep_returns_isometries():
    """Sweep at L = 32, chi = 512 with FP32 products (six products per local solve): its
    truncated sector SVDs reach blocks too large to be held in LDS, so both paths of the
    Jacobi SVD kernel run.  Whichever factored a block, the cores handed back are
    left-orthogonal to rounding, every bond respects chi, and the device energy of the
    returned iterate is the sweep's E_after."""
    from paper_2505_23429_amd.api import Context
    from paper_2505_23429_amd.mpo import build_mpo

    w = S.WORKLOADS[3]
    h, B = S.integrals(w.L, w.n_factors, w.seed)
    mpo = build_mpo(h, B)
    cores, labels = S.random_mps(w.L, w.n_elec, w.two_sz, w.chi, w.seed + 1)
    print(f"L={w.L} chi={w.chi} lengths={w.lengths}", flush=True)
    ctx = Context(chi=w.chi, dav_tol=1e-5, dav_maxiter=6, dav_maxsub=24, matvec_prec="f32")
    ctx.set_mpo(mpo)
    ctx.set_mps(cores, labels)
    rep = ctx.sweep(list(w.lengths))
    c2, l2 = ctx.get_mps()
    assert max(q.shape[0] for q in l2) <= w.chi
    assert max(U.shape[2] for U in c2[:-1]) > 256
    for k, U in enumerate(c2[:-1]):
        M = U.reshape(-1, U.shape[2])
        err = np.abs(M.T @ M - np.eye(M.shape[1])).max()
        assert err < 1e-11, (k, M.shape, err)
    E = ctx.energy()
    assert abs(E - rep["E_after"]) < 1e-9 * abs(E), (E, rep["E_after"])
    ctx.close()



@pytest.mark.timeout(600)
def test_full_size_sweep_blocked_svd_matches_one_workgroup_svd():
    """At L = 32, chi = 512 the wide sector blocks of the splits and of the compression
    (up to about 224 x 141) go to the blocked Jacobi kernels by default.  A converged
    sweep (FP32 products with the FP64 refinement, as timed by the benchmark) gives the
    same coarse eigenvalue and energy after compression with every block on the
    one-workgroup kernel.  The two visit the column pairs in different orders, so they
    agree to rounding wherever the truncation is well conditioned.  Local solves stopped
    early from a random state leave flat spectra at the cut, where a near-degenerate pair
    fixes the kept vector only to eps / gap, so such a sweep is no test of the SVD."""
    from paper_2505_23429_amd.api import Context
    from paper_2505_23429_amd.mpo import build_mpo

    w = S.WORKLOADS[3]
    h, B = S.integrals(w.L, w.n_factors, w.seed)
    mpo = build_mpo(h, B)
    cores, labels = S.random_mps(w.L, w.n_elec, w.two_sz, w.chi, w.seed + 1)
    out = []
    for mode in (1, 0):
        print(f"L={w.L} chi={w.chi} svd_blocked={mode}", flush=True)
        ctx = Context(chi=w.chi, dav_tol=w.dav_tol, dav_maxiter=4000, dav_maxsub=24, matvec_prec="f32",
                      refine_fp64=True, svd_blocked=mode)
        ctx.set_mpo(mpo)
        ctx.set_mps(cores, labels)
        rep = ctx.sweep(list(w.lengths))
        _, l2 = ctx.get_mps()
        assert max(q.shape[0] for q in l2) <= w.chi
        out.append((rep["lambda"], rep["E_after"]))
        print(f"lambda={rep['lambda']:.12f} E_after={rep['E_after']:.12f}", flush=True)
        ctx.close()
    (lam1, e1), (lam0, e0) = out
    assert abs(lam1 - lam0) < 1e-8, (lam1, lam0)
    assert abs(e1 - e0) < 1e-8, (e1, e0)
