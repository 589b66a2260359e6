"""Write the expected values of whole additive two-level sweeps at bench-like sizes.

Run from the repository root:

    python tests/golden/make_sweep_golden.py L12_chi160
    python tests/golden/make_sweep_golden.py L16_chi128
    python tests/golden/make_sweep_golden.py L12_chi160_k2
    python tests/golden/make_sweep_golden.py L12_chi160_1s
    python tests/golden/make_sweep_golden.py L12_chi160_lin

Every value is computed by the environment-chain oracle (``oracle.chain``,
with the oracle's own MPO ``oracle.mpo``) from the seeded inputs of
``seeded_inputs``; nothing comes from the GPU path.  One sweep at these sizes
takes tens of minutes to hours on the CPU, so the results are stored as JSON
fixtures next to this script and the GPU tests compare against them.

Stored per case: the input recipe, <U|H|U> of the normalised input, the
last Ritz value of every subdomain sweep, the coarse overlap and Hamiltonian
matrices, the coarse eigenpair and rank, and <U|H|U> of the compressed next
iterate.  The coarse matrices depend on the sign of each subdomain update
(an eigenvector sign), so they are also stored in the gauge S[0, j] >= 0,
with c then signed so that its largest entry is positive.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import seeded_inputs as S  # noqa: E402
from oracle import chain as CH  # noqa: E402
from oracle import mpo as OM  # noqa: E402
from oracle import tt as T  # noqa: E402

# name: (L, integral seed, chi, TT seed, subdomain lengths, Lanczos tolerance, kept local
# eigenvectors per subdomain (Extension One)[, sites per micro-step (2, or 1: one-site)])
CASES = {
    "L12_chi160": (12, 1012, 160, 23, (4, 4, 4), 1e-11, 1),
    # the L = 16 Hamiltonian of the chi = 256 FP64 workload, at chi = 128 (one oracle
    # sweep at chi = 256 takes about half a day on eight cores)
    "L16_chi128": (16, 1002, 128, 1003, (4, 4, 4, 4), 1e-11, 1),
    # Extension One: the two lowest eigenvectors of every subdomain's last micro-step
    "L12_chi160_k2": (12, 1012, 160, 23, (4, 4, 4), 1e-11, 2),
    # one-site micro-steps (Algorithm 2, one-site branch)
    "L12_chi160_1s": (12, 1012, 160, 23, (4, 4, 4), 1e-11, 1, 1),
}


# linear-system functional (inputs of seeded_inputs.linear_system):
# name: (L, seed, chi, TT seed, subdomain lengths, CG tolerance, bond dimension of F, sites)
CASES_LIN = {
    "L12_chi160_lin": (12, 1012, 160, 23, (4, 4, 4), 1e-12, 32, 2),
}


def run_linear(name):
    L, seed, chi, mps_seed, lengths, tol, chi_f, sites = CASES_LIN[name]
    t0 = time.time()
    hs, B, sigma, F, Fl = S.linear_system(L, L, seed, chi_f)
    mpo = OM.build_mpo(hs, B)
    cores, labels = S.random_mps(L, L, 0, chi, mps_seed)
    cores = S.unit_tt(cores)
    oc = T.left_orthogonalize(cores, labels)

    def log(msg):
        print(f"[{time.time() - t0:8.1f}s] {msg}", flush=True)

    rep = CH.a2dmrg_lin_sweep(mpo, oc, labels, chi, lengths, F, tol=tol, sites=sites, log=log)
    out = {
        "case": name, "functional": "linear", "L": L, "n_elec": L, "two_sz": 0, "seed": seed, "sigma": sigma,
        "chi": chi, "mps_seed": mps_seed, "chi_f": chi_f, "lengths": list(lengths), "cg_tol": tol, "sites": sites,
        "coarse_eps": 1e-8, "svd_cutoff": 1e-12, "tie_rel": 1e-10,
        "J_before": rep.J_before, "E_local": list(map(float, rep.E_local)), "oracle_products": rep.matvecs,
        "S": rep.S.tolist(), "A": rep.A.tolist(), "b": rep.b.tolist(), "c": rep.c.tolist(),
        "J_coarse": rep.J_coarse, "rankS": rep.rankS, "J_after": rep.J_new,
        "bond_dims_after": [int(q.shape[0]) for q in rep.labels], "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"sweep_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    log(f"wrote {path}: J_before={rep.J_before:.12f} J_coarse={rep.J_coarse:.12f} J_after={rep.J_new:.12f}")


def gauge_fix(S_, A_, c):
    """Signs d_j with d_j * S[0, j] >= 0 applied to S, A and c; then the overall
    sign of c that makes its largest entry positive."""
    d = np.sign(S_[0])
    d[0] = 1.0
    d[d == 0] = 1.0
    Sg, Ag, cg = S_ * np.outer(d, d), A_ * np.outer(d, d), c * d
    i = int(np.argmax(np.abs(cg)))
    if cg[i] < 0:
        cg = -cg
    return Sg, Ag, cg


def run(name):
    L, seed, chi, mps_seed, lengths, tol, n_eig = CASES[name][:7]
    sites = CASES[name][7] if len(CASES[name]) > 7 else 2
    t0 = time.time()
    h, B = S.integrals(L, L, seed)
    mpo = OM.build_mpo(h, B)
    cores, labels = S.random_mps(L, L, 0, chi, mps_seed)
    oc = T.left_orthogonalize(cores, labels)

    def log(msg):
        print(f"[{time.time() - t0:8.1f}s] {msg}", flush=True)

    rep = CH.a2dmrg_sweep(mpo, oc, labels, chi, lengths, tol=tol, log=log, n_eig=n_eig, sites=sites)
    Sg, Ag, cg = gauge_fix(rep.S, rep.A, rep.c)
    out = {
        "case": name, "L": L, "n_elec": L, "two_sz": 0, "integral_seed": seed, "n_factors": L, "chi": chi,
        "mps_seed": mps_seed, "lengths": list(lengths), "lanczos_tol": tol, "coarse_k": n_eig, "sites": sites, "coarse_eps": 1e-8,
        "svd_cutoff": 1e-12, "tie_rel": 1e-10,
        "E_before": rep.E_before, "E_local": list(map(float, rep.E_local)), "oracle_products": rep.matvecs,
        "S": rep.S.tolist(), "A": rep.A.tolist(), "S_gauge": Sg.tolist(), "A_gauge": Ag.tolist(),
        "c_gauge": cg.tolist(), "lambda": rep.lam, "rankS": rep.rankS, "E_after": rep.E_new,
        "bond_dims_after": [int(q.shape[0]) for q in rep.labels], "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"sweep_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    log(f"wrote {path}: E_before={rep.E_before:.12f} lambda={rep.lam:.12f} E_after={rep.E_new:.12f}")


if __name__ == "__main__":
    for n in sys.argv[1:] or sorted(CASES) + sorted(CASES_LIN):
        run_linear(n) if n in CASES_LIN else run(n)
