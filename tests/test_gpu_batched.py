"""Concurrent subdomain solves (Step 2 of Algorithm 2: the local problems of the
subdomains are independent).  Running them on several workers, each a host
thread with its own HIP stream, must give exactly the result of running them
one after another on the context's stream: every kernel is deterministic and a
subdomain's solve reads only the Step-1 cores and environments."""
import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu


def _run(mpo, cores, labels, lengths, workers, **kw):
    from paper_2505_23429_amd.api import open_context

    ctx = open_context(mpo, cores, labels, sub_workers=workers, **kw)
    rep = ctx.sweep(list(lengths))
    out, lab = ctx.get_mps()
    ctx.close()
    return rep, out, lab


@pytest.mark.parametrize("prec,refine", [("f64", False), ("f32", True)])
def test_concurrent_solves_equal_sequential(prec, refine):
    from paper_2505_23429_amd.mpo import build_mpo

    L, chi, lengths = 12, 48, (2, 4, 3, 3)
    h, B = S.integrals(L, L, 1012)
    mpo = build_mpo(h, B)
    cores, labels = S.random_mps(L, L, 0, chi, 51)
    kw = dict(chi=chi, dav_tol=1e-8, matvec_prec=prec, refine_fp64=refine)
    print(f"L={L} chi={chi} lengths={lengths} prec={prec}", flush=True)
    r1, c1, l1 = _run(mpo, cores, labels, lengths, 1, **kw)
    r4, c4, l4 = _run(mpo, cores, labels, lengths, 4, **kw)
    assert list(r1["matvecs"]) == list(r4["matvecs"])
    assert np.array_equal(r1["E_local"], r4["E_local"])
    assert np.array_equal(r1["S"], r4["S"]) and np.array_equal(r1["A"], r4["A"])
    assert np.array_equal(r1["c"], r4["c"])
    assert r1["E_after"] == r4["E_after"]
    for a, b in zip(c1, c4):
        assert a.shape == b.shape and np.array_equal(a, b)
    for a, b in zip(l1, l4):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    # more workers than subdomains, and a one-site last subdomain
    r8, _, _ = _run(mpo, cores, labels, (4, 4, 3, 1), 8, **kw)
    r1b, _, _ = _run(mpo, cores, labels, (4, 4, 3, 1), 1, **kw)
    assert np.array_equal(r8["E_local"], r1b["E_local"]) and r8["E_after"] == r1b["E_after"]


def test_worker_out_of_memory_recovers_with_the_same_result():
    """A worker whose task cannot get device memory frees its workspaces and leaves; the
    tasks it gave up, and any no worker started, run again one after another on the
    context.  Forced here from the host with a one-byte allocation limit per worker task
    (every worker fails at its first allocation), the sweep must equal the one-worker
    sweep bit for bit."""
    from paper_2505_23429_amd.mpo import build_mpo

    L, chi, lengths = 12, 48, (2, 4, 3, 3)
    h, B = S.integrals(L, L, 1012)
    mpo = build_mpo(h, B)
    cores, labels = S.random_mps(L, L, 0, chi, 51)
    kw = dict(chi=chi, dav_tol=1e-8, matvec_prec="f64")
    print(f"L={L} chi={chi} lengths={lengths} worker allocation limit 1 byte", flush=True)
    r1, c1, l1 = _run(mpo, cores, labels, lengths, 1, **kw)
    r4, c4, l4 = _run(mpo, cores, labels, lengths, 4, worker_alloc_limit=1, **kw)
    assert list(r1["matvecs"]) == list(r4["matvecs"])
    assert np.array_equal(r1["E_local"], r4["E_local"])
    assert np.array_equal(r1["S"], r4["S"]) and np.array_equal(r1["A"], r4["A"])
    assert r1["E_after"] == r4["E_after"]
    for a, b in zip(c1, c4):
        assert a.shape == b.shape and np.array_equal(a, b)
