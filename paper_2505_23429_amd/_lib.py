"""ctypes loader of the in-tree HIP library ``libtt.so`` (declared in include/tt.h).

Argument marshalling only.  Importing this module fails loudly when the library
has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtt.so")

TT_OK, TT_WNOCONV, TT_WRANKDEF = 0, 1, 2
TT_EINVAL, TT_ESTATE, TT_ENOMEM, TT_EHIP, TT_EINTERNAL = -1, -2, -3, -4, -5
TT_F64, TT_F32, TT_BF16 = 0, 1, 2
TT_MAX_SUB = 64

# every entry point declared in include/tt.h
EXPORTS = (
    "tt_default_opts", "tt_create", "tt_destroy", "tt_last_error", "tt_set_mpo", "tt_set_mps", "tt_get_mps",
    "tt_energy", "tt_local_solve", "tt_coarse_correct", "tt_sweep", "tt_dmrg2", "tt_heff_apply_dev",
    "tt_env_update_dev", "tt_heff_energy_grad_dev", "tt_energy_mpo_grad", "tt_gemm_dev", "tt_kernel_timing",
    "tt_window_apply_dev", "tt_mps_checkpoint", "tt_heff_apply_dev_noalloc", "tt_set_rhs", "tt_functional",
)
TT_NOALLOC_SCRATCH_BYTES = 256 << 20


class Opts(C.Structure):
    _fields_ = [
        ("chi_max", C.c_int), ("svd_cutoff", C.c_double), ("tie_rel", C.c_double), ("dav_tol", C.c_double),
        ("dav_maxiter", C.c_int), ("dav_maxsub", C.c_int), ("coarse_eps", C.c_double), ("matvec_prec", C.c_int),
        ("refine_fp64", C.c_int), ("lowprec_tol", C.c_double), ("device", C.c_int), ("qn_skip", C.c_int),
        ("sub_workers", C.c_int), ("mix_stage", C.c_int), ("svd_lds", C.c_int),
        ("worker_alloc_limit", C.c_longlong), ("stream", C.c_void_p), ("dev_alloc", C.c_void_p),
        ("dev_free", C.c_void_p), ("alloc_user", C.c_void_p), ("coarse_k", C.c_int),
        ("one_site", C.c_int), ("functional", C.c_int), ("coarse_krylov", C.c_int),
        ("graph_products", C.c_int), ("precontract", C.c_int), ("svd_blocked", C.c_int),
    ]


# tt_opts.dev_alloc / dev_free callback types
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


_N = (TT_MAX_SUB + 1) * (TT_MAX_SUB + 1)


class SweepReport(C.Structure):
    _fields_ = [
        ("nsub", C.c_int), ("E_before", C.c_double), ("E_local", C.c_double * TT_MAX_SUB),
        ("matvecs", C.c_int * TT_MAX_SUB), ("S", C.c_double * _N), ("A", C.c_double * _N),
        ("coef", C.c_double * (TT_MAX_SUB + 1)), ("lambda_", C.c_double), ("rankS", C.c_int),
        ("E_after", C.c_double), ("discarded", C.c_double), ("seconds", C.c_double * 4),
        ("flops_heff", C.c_double), ("seconds_heff", C.c_double), ("phase_seconds", C.c_double * 9),
        ("matvecs_f64", C.c_int * TT_MAX_SUB), ("nstates", C.c_int), ("rhs", C.c_double * (TT_MAX_SUB + 1)),
        ("coarse_matvecs", C.c_int),
    ]


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build() or "
            "python -m paper_2505_23429_amd.build)")
    lib = C.CDLL(LIB_PATH)
    P, I, D, VP = C.POINTER, C.c_int, C.c_double, C.c_void_p
    lib.tt_default_opts.argtypes = [P(Opts)]
    lib.tt_default_opts.restype = None
    lib.tt_create.argtypes = [P(Opts), P(VP)]
    lib.tt_create.restype = I
    lib.tt_destroy.argtypes = [VP]
    lib.tt_destroy.restype = None
    lib.tt_last_error.argtypes = [VP]
    lib.tt_last_error.restype = C.c_char_p
    lib.tt_set_mpo.argtypes = [VP, I, P(I), P(I), P(P(C.c_int32)), P(P(C.c_int32)), P(P(D)), P(P(C.c_int32)), P(I)]
    lib.tt_set_mpo.restype = I
    lib.tt_set_mps.argtypes = [VP, I, P(I), P(P(D)), P(P(C.c_int32))]
    lib.tt_set_mps.restype = I
    lib.tt_get_mps.argtypes = [VP, P(I), P(P(D)), P(P(C.c_int32))]
    lib.tt_get_mps.restype = I
    lib.tt_energy.argtypes = [VP, P(D)]
    lib.tt_energy.restype = I
    lib.tt_set_rhs.argtypes = [VP, I, P(I), P(P(D)), P(P(C.c_int32))]
    lib.tt_set_rhs.restype = I
    lib.tt_functional.argtypes = [VP, P(D)]
    lib.tt_functional.restype = I
    lib.tt_local_solve.argtypes = [VP, I, P(I), P(D), P(I)]
    lib.tt_local_solve.restype = I
    lib.tt_coarse_correct.argtypes = [VP, P(D), P(D), P(D), P(D), P(D), P(I)]
    lib.tt_coarse_correct.restype = I
    lib.tt_sweep.argtypes = [VP, I, P(I), P(SweepReport)]
    lib.tt_sweep.restype = I
    lib.tt_dmrg2.argtypes = [VP, I, P(D)]
    lib.tt_dmrg2.restype = I
    lib.tt_heff_apply_dev.argtypes = [VP, I, I, I, I, I, I, VP, VP, I, P(C.c_int32), P(C.c_int32), P(D), I,
                                      P(C.c_int32), P(C.c_int32), P(D), VP, VP]
    lib.tt_heff_apply_dev.restype = I
    lib.tt_heff_apply_dev_noalloc.argtypes = lib.tt_heff_apply_dev.argtypes
    lib.tt_heff_apply_dev_noalloc.restype = I
    lib.tt_mps_checkpoint.argtypes = [VP, I]
    lib.tt_mps_checkpoint.restype = I
    lib.tt_window_apply_dev.argtypes = [VP, I, I, I, P(C.c_int32), P(C.c_int32), VP, VP, I, VP, VP]
    lib.tt_window_apply_dev.restype = I
    lib.tt_env_update_dev.argtypes = [VP, I, I, I, I, I, I, I, VP, VP, VP, I, P(C.c_int32), P(C.c_int32), P(D), VP]
    lib.tt_env_update_dev.restype = I
    lib.tt_heff_energy_grad_dev.argtypes = [VP, I, I, I, I, I, VP, VP, I, P(C.c_int32), P(C.c_int32), P(D), I,
                                            P(C.c_int32), P(C.c_int32), P(D), VP, P(D), VP, VP, VP, P(D), P(D)]
    lib.tt_heff_energy_grad_dev.restype = I
    lib.tt_gemm_dev.argtypes = [VP, I, I, I, I, I, I, P(C.c_longlong), I, I, D, D, VP, VP, VP]
    lib.tt_gemm_dev.restype = I
    lib.tt_kernel_timing.argtypes = [VP, I, P(D), I]
    lib.tt_kernel_timing.restype = I
    lib.tt_energy_mpo_grad.argtypes = [VP, P(D), P(P(D))]
    lib.tt_energy_mpo_grad.restype = I
    _lib = lib
    return lib
