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
