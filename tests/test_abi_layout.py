"""The ctypes mirrors of the C-ABI structs (tt_opts, tt_sweep_report) have the layout
the C compiler gives the declarations in include/tt.h: every field at the same offset,
and the same total size.  Compiles a small C program with gcc (no GPU)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _c_layout(tmp_path, struct, fields):
    src = tmp_path / "layout.c"
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "tt.h"', "int main(void) {",
             f'  printf("size %zu\\n", sizeof({struct}));']
    lines += [f'  printf("{f} %zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    return {k: int(v) for k, v in (ln.split() for ln in out if ln.strip())}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("which", ["opts", "report"])
def test_ctypes_structs_match_the_header(tmp_path, which):
    from paper_2505_23429_amd import _lib as L

    cls, struct = (L.Opts, "tt_opts") if which == "opts" else (L.SweepReport, "tt_sweep_report")
    names = [f[0] for f in cls._fields_]
    cnames = ["lambda" if n == "lambda_" else n for n in names]
    lay = _c_layout(tmp_path, struct, cnames)
    assert lay["size"] == C.sizeof(cls)
    for n, cn in zip(names, cnames):
        assert lay[cn] == getattr(cls, n).offset, (n, lay[cn], getattr(cls, n).offset)
