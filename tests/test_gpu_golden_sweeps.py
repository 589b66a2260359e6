"""Whole additive two-level sweeps at bench-like sizes against the environment-chain
oracle (stored expected values under tests/golden/, written by
make_sweep_golden.py from oracle/ only).

From the same seeded Hamiltonian and chi-saturated random tensor train, the
library's sweep (its own MPO, block-sparse products, Davidson, Jacobi SVD,
coarse step, compression) must reproduce the oracle's:
* FP64 products: |dE| <= 1e-8 Ha for <U|H|U> before and after, every
  subdomain's last Ritz value and the coarse eigenvalue; the coarse overlap and
  Hamiltonian entry by entry and the coarse coefficients with their signs, in
  the gauge S[0, j] >= 0;
* FP32 and bfloat16 products with FP64 refinement: |dE| <= 1e-6 Ha.
"""
import json
import os

import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu
HERE = os.path.join(os.path.dirname(__file__), "golden")


def _gauge(S_, A_, c):
    d = np.sign(S_[0])
    d[0] = 1.0
    d[d == 0] = 1.0
    Sg, Ag, cg = S_ * np.outer(d, d), A_ * np.outer(d, d), c * d
    i = int(np.argmax(np.abs(cg)))
    return Sg, Ag, (-cg if cg[i] < 0 else cg)


def _run(name, prec):
    from paper_2505_23429_amd.api import Context
    from paper_2505_23429_amd.mpo import build_mpo

    g = json.load(open(os.path.join(HERE, f"sweep_{name}.json")))
    L, chi = g["L"], g["chi"]
    h, B = S.integrals(L, g["n_factors"], g["integral_seed"])
    cores, labels = S.random_mps(L, g["n_elec"], g["two_sz"], chi, g["mps_seed"])
    print(f"{name} {prec}: L={L} chi={chi} lengths={g['lengths']}", flush=True)
    kw = dict(chi=chi, dav_tol=1e-11, dav_maxiter=2000, coarse_eps=g["coarse_eps"], svd_cutoff=g["svd_cutoff"],
              tie_rel=g["tie_rel"])
    if prec != "f64":
        kw.update(matvec_prec=prec, refine_fp64=True, lowprec_tol=1e-5)
    ctx = Context(**kw)
    ctx.set_mpo(build_mpo(h, B))
    ctx.set_mps(cores, labels)
    rep = ctx.sweep(list(g["lengths"]))
    _, l2 = ctx.get_mps()
    ctx.close()
    print(f"  E_after {rep['E_after']:.12f} (oracle {g['E_after']:.12f}), products {list(rep['matvecs'])}", flush=True)
    return g, rep, l2


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["L12_chi160", "L16_chi128"])
def test_fp64_sweep_matches_oracle(name):
    g, rep, l2 = _run(name, "f64")
    assert rep["status"] in (0, 2)  # every local solve converged (no TT_WNOCONV)
    assert abs(rep["E_before"] - g["E_before"]) < 1e-10
    assert np.abs(rep["E_local"] - np.array(g["E_local"])).max() < 1e-8
    Sg, Ag, cg = _gauge(rep["S"], rep["A"], rep["c"])
    assert np.abs(Sg - np.array(g["S_gauge"])).max() < 1e-9
    assert np.abs(Ag - np.array(g["A_gauge"])).max() < 1e-8
    assert np.abs(cg - np.array(g["c_gauge"])).max() < 1e-7
    assert rep["rankS"] == g["rankS"]
    assert abs(rep["lambda"] - g["lambda"]) < 1e-8
    assert abs(rep["E_after"] - g["E_after"]) < 1e-8
    assert [q.shape[0] for q in l2] == g["bond_dims_after"]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_precision_sweep_matches_oracle(prec):
    g, rep, _ = _run("L12_chi160", prec)
    assert rep["status"] in (0, 2)
    assert np.abs(rep["E_local"] - np.array(g["E_local"])).max() < 1e-6
    assert abs(rep["lambda"] - g["lambda"]) < 1e-6
    assert abs(rep["E_after"] - g["E_after"]) < 1e-6
