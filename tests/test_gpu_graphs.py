"""Products replayed from HIP graphs (tt_opts.graph_products): every local problem's
block-sparse products after the second one are replays of a captured graph, with the
host's Rayleigh-Ritz work and synchronisations between replays.  The whole sweep must
equal the eagerly launched one bit for bit (same kernels, same order), in FP64, FP32
and bf16 with the FP64-anchored refinement (whose products alternate precisions)."""
import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu


def _sweep(L, seed, chi, lengths, mps_seed, prec, refine, graphs, workers):
    from paper_2505_23429_amd.api import open_context
    from paper_2505_23429_amd.mpo import build_mpo

    h, B = S.integrals(L, L, seed)
    cores, labels = S.random_mps(L, L, 0, chi, mps_seed)
    ctx = open_context(build_mpo(h, B), cores, labels, chi=chi, dav_tol=1e-10, dav_maxiter=2000, matvec_prec=prec,
                       refine_fp64=refine, graph_products=graphs, sub_workers=workers)
    rep = ctx.sweep(list(lengths))
    c2, l2 = ctx.get_mps()
    ctx.close()
    return rep, c2


@pytest.mark.parametrize("L,seed,chi,lengths,mps_seed,prec,refine,workers",
                         [(8, 1008, 24, (2, 3, 3), 27, "f64", False, 1),
                          (8, 1008, 24, (2, 3, 3), 27, "f32", True, 1),
                          (8, 1008, 24, (2, 3, 3), 27, "bf16", True, 1),
                          (12, 1012, 160, (4, 4, 4), 23, "f32", True, 3)])
def test_graph_products_equal_eager_launches(L, seed, chi, lengths, mps_seed, prec, refine, workers):
    print(f"graph products L={L} chi={chi} prec={prec} refine={refine} workers={workers}", flush=True)
    r0, c0 = _sweep(L, seed, chi, lengths, mps_seed, prec, refine, False, workers)
    r1, c1 = _sweep(L, seed, chi, lengths, mps_seed, prec, refine, True, workers)
    assert int(np.sum(r1["matvecs"])) > 4 * len(lengths)  # replays happened
    for k in ("E_before", "lambda", "E_after"):
        assert r0[k] == r1[k], k
    for k in ("E_local", "matvecs", "matvecs_f64", "S", "A", "c"):
        assert np.array_equal(r0[k], r1[k]), k
    assert all(np.array_equal(a, b) for a, b in zip(c0, c1))
