"""Step 3 by Krylov iterations without forming the coarse Hamiltonian matrix
(products through the structured combination W(v) = sum_j v_j U^j): the same
coarse eigenpair and next iterate as the explicit coarse matrices, against the
dense-vector oracle at L = 6, 8 (two-site, one-site, Extension One) and against the
environment-chain oracle's stored values at L = 12, chi = 160."""
import json
import os

import numpy as np
import pytest

import seeded_inputs as S
from oracle import tt as T

pytestmark = pytest.mark.gpu
HERE = os.path.join(os.path.dirname(__file__), "golden")


def _gauge(S_, c):
    d = np.sign(S_[0])
    d[0] = 1.0
    d[d == 0] = 1.0
    cg = c * d
    i = int(np.argmax(np.abs(cg)))
    return -cg if cg[i] < 0 else cg


@pytest.mark.parametrize("L,seed,chi,lengths,mps_seed,K,sites",
                         [(6, 1001, 16, (2, 2, 2), 19, 1, 2), (8, 1008, 24, (2, 3, 3), 27, 1, 2),
                          (8, 1008, 16, (3, 3, 2), 19, 2, 2), (8, 1008, 24, (3, 1, 4), 27, 1, 1),
                          (6, 1006, 12, (1, 1, 1, 1, 1, 1), 21, 1, 1)])
def test_krylov_coarse_step_matches_explicit_and_oracle(L, seed, chi, lengths, mps_seed, K, sites):
    from paper_2505_23429_amd.api import open_context
    from paper_2505_23429_amd.mpo import build_mpo

    h, B = S.integrals(L, L, seed)
    cores, labels = S.random_mps(L, L, 0, chi, mps_seed)
    prob = T.Problem(h, B, L, 0)
    oc = T.left_orthogonalize(cores, labels)
    print(f"krylov coarse step L={L} seed={seed} chi={chi} lengths={lengths} K={K} sites={sites}", flush=True)
    reps = []
    for kry in (False, True):
        ctx = open_context(build_mpo(h, B), cores, labels, chi=chi, dav_tol=1e-10, coarse_k=K, one_site=sites == 1,
                           coarse_krylov=kry)
        reps.append((ctx.sweep(list(lengths)), ctx.get_mps()))
        ctx.close()
    (rx, (cx, lx)), (rk, (ck, lk)) = reps
    assert np.isnan(rk["A"]).all() and not np.isnan(rx["A"]).any()
    assert 1 <= rk["coarse_matvecs"] <= rk["rankS"] and rx["coarse_matvecs"] == 0
    assert np.abs(rk["S"] - rx["S"]).max() < 1e-12
    assert abs(rk["lambda"] - rx["lambda"]) < 1e-10
    assert np.abs(rk["c"] - rx["c"]).max() < 1e-7
    assert abs(rk["E_after"] - rx["E_after"]) < 1e-10
    assert [q.shape[0] for q in lk] == [q.shape[0] for q in lx]
    ro = T.a2dmrg_sweep(prob, oc, labels, chi, lengths, n_eig=K, sites=sites)
    assert abs(rk["lambda"] - ro.lam) < 1e-8
    assert np.abs(_gauge(rk["S"], rk["c"]) - _gauge(ro.S, ro.c)).max() < 1e-7
    assert abs(rk["E_after"] - ro.E_new) < 1e-8


@pytest.mark.timeout(900)
def test_krylov_coarse_step_L12_matches_stored_oracle():
    from paper_2505_23429_amd.api import Context
    from paper_2505_23429_amd.mpo import build_mpo

    g = json.load(open(os.path.join(HERE, "sweep_L12_chi160.json")))
    L, chi = g["L"], g["chi"]
    h, B = S.integrals(L, g["n_factors"], g["integral_seed"])
    cores, labels = S.random_mps(L, g["n_elec"], g["two_sz"], chi, g["mps_seed"])
    ctx = Context(chi=chi, dav_tol=1e-11, dav_maxiter=2000, coarse_krylov=True)
    ctx.set_mpo(build_mpo(h, B))
    ctx.set_mps(cores, labels)
    rep = ctx.sweep(list(g["lengths"]))
    _, l2 = ctx.get_mps()
    ctx.close()
    print(f"lambda {rep['lambda']:.12f} (oracle {g['lambda']:.12f}), coarse products {rep['coarse_matvecs']}", flush=True)
    assert rep["status"] in (0, 2)
    assert np.abs(_gauge(rep["S"], rep["c"]) - np.array(g["c_gauge"])).max() < 1e-7
    assert abs(rep["lambda"] - g["lambda"]) < 1e-8
    assert abs(rep["E_after"] - g["E_after"]) < 1e-8
    assert [q.shape[0] for q in l2] == g["bond_dims_after"]
