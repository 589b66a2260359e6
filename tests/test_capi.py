"""The C-ABI library loads and exports every symbol that include/tt.h declares;
host-side validation rejects bad input before any device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tt_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2505_23429_amd import _lib

    lib = _lib.load()
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_default_options_and_invalid_create():
    from paper_2505_23429_amd import _lib

    lib = _lib.load()
    o = _lib.Opts()
    lib.tt_default_opts(C.byref(o))
    assert o.chi_max > 0 and o.svd_cutoff == 1e-12 and o.tie_rel == 1e-10
    h = C.c_void_p()
    bad = _lib.Opts()
    lib.tt_default_opts(C.byref(bad))
    bad.dav_maxsub = 1
    assert lib.tt_create(C.byref(bad), C.byref(h)) == _lib.TT_EINVAL
    assert lib.tt_create(None, C.byref(h)) == _lib.TT_EINVAL
    assert lib.tt_last_error(None) == b"null context"


@pytest.mark.parametrize("field,value", [
    ("chi_max", 0), ("dav_maxiter", 0), ("dav_maxsub", 3), ("matvec_prec", 3), ("matvec_prec", -1),
    ("sub_workers", -1), ("sub_workers", 65), ("mix_stage", 3), ("mix_stage", -1), ("svd_lds", 2),
    ("worker_alloc_limit", -1), ("coarse_k", 0), ("coarse_k", 9), ("one_site", 2), ("one_site", -1),
    ("functional", 2), ("functional", -1), ("coarse_krylov", 2), ("coarse_krylov", -1),
    ("graph_products", 2), ("graph_products", -1), ("precontract", 3), ("precontract", -1),
    ("svd_blocked", 5), ("svd_blocked", -1),
])
def test_create_rejects_each_invalid_option(field, value):
    """tt_create validates the options before it touches the device: every value outside
    its documented range is refused with TT_EINVAL and no context."""
    from paper_2505_23429_amd import _lib

    lib = _lib.load()
    o = _lib.Opts()
    lib.tt_default_opts(C.byref(o))
    assert (o.mix_stage, o.svd_lds, o.worker_alloc_limit, o.sub_workers, o.svd_blocked) == (0, 1, 0, 0, 1)
    setattr(o, field, value)
    h = C.c_void_p()
    assert lib.tt_create(C.byref(o), C.byref(h)) == _lib.TT_EINVAL
    assert not h.value


@pytest.mark.parametrize("field,value", [("matvec_prec", 1), ("matvec_prec", 2), ("qn_skip", 0)])
def test_one_site_needs_fp64_block_sparse_products(field, value):
    """One-site micro-steps run the FP64 block-sparse one-site product only: any other
    product setting is refused at tt_create (before the device is touched)."""
    from paper_2505_23429_amd import _lib

    lib = _lib.load()
    o = _lib.Opts()
    lib.tt_default_opts(C.byref(o))
    assert (o.one_site, o.coarse_k) == (0, 1)
    o.one_site = 1
    setattr(o, field, value)
    h = C.c_void_p()
    assert lib.tt_create(C.byref(o), C.byref(h)) == _lib.TT_EINVAL
    assert not h.value


@pytest.mark.parametrize("field,value", [("matvec_prec", 1), ("matvec_prec", 2), ("qn_skip", 0), ("coarse_k", 2),
                                         ("coarse_krylov", 1)])
def test_linear_functional_needs_fp64_block_sparse_products(field, value):
    """The linear-system functional solves its micro-steps by FP64 conjugate gradients
    on the block-sparse product and has no several-eigenvector or Krylov-coarse variant."""
    from paper_2505_23429_amd import _lib

    lib = _lib.load()
    o = _lib.Opts()
    lib.tt_default_opts(C.byref(o))
    assert o.functional == 0
    o.functional = 1
    setattr(o, field, value)
    h = C.c_void_p()
    assert lib.tt_create(C.byref(o), C.byref(h)) == _lib.TT_EINVAL
    assert not h.value
