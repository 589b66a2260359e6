"""Python binding with the names of the C ABI (include/tt.h).

Argument marshalling only: every step of the additive two-level DMRG path runs
in the HIP library.  PyTorch supplies device memory for the kernel-level entry
points; the context owns its own device state.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

PREC = {"f64": L.TT_F64, "f32": L.TT_F32, "bf16": L.TT_BF16}


class TTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tt error {code}: {msg}")
        self.code = code


def _ptr_array(arrs, ctype):
    keep = [np.ascontiguousarray(a, dtype=np.dtype(ctype)) for a in arrs]
    arr = (C.POINTER(ctype) * len(keep))(*[a.ctypes.data_as(C.POINTER(ctype)) for a in keep])
    return arr, keep


def _iarr(v):
    v = np.ascontiguousarray(v, dtype=np.int32)
    return v, v.ctypes.data_as(C.POINTER(C.c_int))


class Context:
    """One device context: MPO, current TT iterate, environment caches."""

    def __init__(self, chi=64, dav_tol=1e-8, dav_maxiter=200, dav_maxsub=24, coarse_eps=1e-8, svd_cutoff=1e-12,
                 tie_rel=1e-10, matvec_prec="f64", refine_fp64=False, lowprec_tol=1e-5, device=0, qn_skip=True,
                 sub_workers=0, mix_stage=0, svd_lds=True, worker_alloc_limit=0):
        self.lib = L.load()
        o = L.Opts()
        self.lib.tt_default_opts(C.byref(o))
        o.chi_max = chi
        o.dav_tol = dav_tol
        o.dav_maxiter = dav_maxiter
        o.dav_maxsub = dav_maxsub
        o.coarse_eps = coarse_eps
        o.svd_cutoff = svd_cutoff
        o.tie_rel = tie_rel
        o.matvec_prec = PREC[matvec_prec] if isinstance(matvec_prec, str) else int(matvec_prec)
        o.refine_fp64 = int(bool(refine_fp64))
        o.lowprec_tol = lowprec_tol
        o.device = device
        o.qn_skip = int(bool(qn_skip))
        o.sub_workers = int(sub_workers)
        o.mix_stage = int(mix_stage)
        o.svd_lds = int(bool(svd_lds))
        o.worker_alloc_limit = int(worker_alloc_limit)
        self.opts = o
        h = C.c_void_p()
        rc = self.lib.tt_create(C.byref(o), C.byref(h))
        if rc != 0:
            raise TTError(rc, "context creation failed")
        self.h = h
        self.last_status = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.tt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        self.last_status = rc
        if rc < 0:
            raise TTError(rc, self.lib.tt_last_error(self.h).decode())
        return rc

    # ---- problem setup -------------------------------------------------
    def set_mpo(self, mpo):
        Lsites = mpo.L
        R, Rp = _iarr(mpo.R)
        nnz, nnzp = _iarr([len(a) for a in mpo.A])
        A, ka = _ptr_array(mpo.A, C.c_int32)
        B, kb = _ptr_array(mpo.B, C.c_int32)
        ops, ko = _ptr_array([o.reshape(-1) for o in mpo.ops], C.c_double)
        cq, kq = _ptr_array([q.reshape(-1) for q in mpo.chan_q], C.c_int32)
        blocks = getattr(mpo, "blocks", None)
        blk = np.asarray(blocks if blocks is not None else [(-1, -1, -1, -1)] * Lsites, dtype=np.int32).reshape(-1)
        blk, blkp = _iarr(blk)
        self._check(self.lib.tt_set_mpo(self.h, Lsites, Rp, nnzp, A, B, ops, cq, blkp))

    def set_mps(self, cores, labels):
        Lsites = len(cores)
        r, rp = _iarr([c.shape[0] for c in cores] + [cores[-1].shape[2]])
        U, ku = _ptr_array([c.reshape(-1) for c in cores], C.c_double)
        q, kq = _ptr_array([np.asarray(l).reshape(-1) for l in labels], C.c_int32)
        self._check(self.lib.tt_set_mps(self.h, Lsites, rp, U, q))
        self._L = Lsites

    def get_mps(self):
        # size query
        Lsites = self._length()
        r = np.zeros(Lsites + 1, dtype=np.int32)
        self._check(self.lib.tt_get_mps(self.h, r.ctypes.data_as(C.POINTER(C.c_int)), None, None))
        cores = [np.zeros((r[k], 4, r[k + 1])) for k in range(Lsites)]
        labels = [np.zeros((r[k], 2), dtype=np.int32) for k in range(Lsites + 1)]
        U, ku = _ptr_array([c.reshape(-1) for c in cores], C.c_double)
        q, kq = _ptr_array([l.reshape(-1) for l in labels], C.c_int32)
        self._check(self.lib.tt_get_mps(self.h, r.ctypes.data_as(C.POINTER(C.c_int)), U, q))
        cores = [ku[k].reshape(r[k], 4, r[k + 1]) for k in range(Lsites)]
        labels = [kq[k].reshape(r[k], 2) for k in range(Lsites + 1)]
        return cores, labels

    def _length(self):
        if not hasattr(self, "_L"):
            raise RuntimeError("set_mps first")
        return self._L

    def energy(self):
        e = C.c_double()
        self._check(self.lib.tt_energy(self.h, C.byref(e)))
        return e.value

    # ---- the additive two-level iteration --------------------------------
    def local_solve(self, lengths):
        n = len(lengths)
        lp, lpp = _iarr(lengths)
        E = np.zeros(n)
        mv = np.zeros(n, dtype=np.int32)
        rc = self._check(self.lib.tt_local_solve(self.h, n, lpp, E.ctypes.data_as(C.POINTER(C.c_double)),
                                                 mv.ctypes.data_as(C.POINTER(C.c_int))))
        return E, mv, rc

    def coarse_correct(self, nsub):
        n = nsub + 1
        S = np.zeros((n, n))
        A = np.zeros((n, n))
        c = np.zeros(n)
        lam = C.c_double()
        E = C.c_double()
        rank = C.c_int()
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        rc = self._check(self.lib.tt_coarse_correct(self.h, dp(S), dp(A), dp(c), C.byref(lam), C.byref(E),
                                                    C.byref(rank)))
        return {"S": S, "A": A, "c": c, "lambda": lam.value, "E": E.value, "rankS": rank.value, "status": rc}

    def sweep(self, lengths):
        n = len(lengths)
        lp, lpp = _iarr(lengths)
        rep = L.SweepReport()
        rc = self._check(self.lib.tt_sweep(self.h, n, lpp, C.byref(rep)))
        m = n + 1
        S = np.array(rep.S[: m * m]).reshape(m, m)
        A = np.array(rep.A[: m * m]).reshape(m, m)
        return {
            "status": rc, "E_before": rep.E_before, "E_local": np.array(rep.E_local[:n]),
            "matvecs": np.array(rep.matvecs[:n]), "S": S, "A": A, "c": np.array(rep.coef[:m]),
            "lambda": rep.lambda_, "rankS": rep.rankS, "E_after": rep.E_after, "discarded": rep.discarded,
            "seconds": list(rep.seconds), "flops_heff": rep.flops_heff, "seconds_heff": rep.seconds_heff,
            "phase_seconds": list(rep.phase_seconds),
        }

    def checkpoint(self, restore=False):
        """Keep a device copy of the current iterate, or make the kept copy current again."""
        self._check(self.lib.tt_mps_checkpoint(self.h, 1 if restore else 0))

    def dmrg2(self, nsweeps):
        E = np.zeros(2 * nsweeps)
        rc = self._check(self.lib.tt_dmrg2(self.h, nsweeps, E.ctypes.data_as(C.POINTER(C.c_double))))
        return E, rc

    KERNELS = ("gemm_Lx", "mix1_gather", "mix1_heavy_gemm", "mix1_heavy_scatter", "mix2_gather",
               "mix2_heavy_gemm", "mix2_heavy_scatter", "gemm_R", "gemm_R_reduce")

    def kernel_timing(self, enable=True, reset=False):
        """Per-kernel stats of the products: one row per entry of KERNELS,
        columns (ms, launches, algorithmic flops, algorithmic bytes)."""
        n = len(self.KERNELS)
        st = np.zeros(4 * n)
        self._check(self.lib.tt_kernel_timing(self.h, int(enable), st.ctypes.data_as(C.POINTER(C.c_double)),
                                              int(reset)))
        return st.reshape(n, 4)

    def mpo_gradient(self, mpo):
        """dE/dW for every MPO entry of E = <U|H|U> (normalised current iterate)."""
        g = [np.zeros((len(a), 16)) for a in mpo.A]
        G, kg = _ptr_array([x.reshape(-1) for x in g], C.c_double)
        E = C.c_double()
        self._check(self.lib.tt_energy_mpo_grad(self.h, C.byref(E), G))
        return E.value, [kg[k].reshape(-1, 4, 4) for k in range(len(g))]


def open_context(mpo, cores, labels, **kw):
    ctx = Context(**kw)
    ctx.set_mpo(mpo)
    ctx._L = mpo.L
    ctx.set_mps(cores, labels)
    return ctx


# ---- kernel-level entry points (device tensors from torch) -------------------

def _sparse(W):
    A, B, ops = W
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    ops = np.ascontiguousarray(ops, dtype=np.float64).reshape(-1)
    return A, B, ops


def heff_apply(ctx, prec, Lenv, W1, W2, Renv, x, y=None):
    """y = H_eff x with torch device tensors Lenv [RA][rl][rl], Renv [RC][rr][rr], x [rl][4][4][rr]."""
    import torch

    RA, rl, _ = Lenv.shape
    RC, rr, _ = Renv.shape
    A1, B1, o1 = _sparse(W1)
    A2, B2, o2 = _sparse(W2)
    RB = int(max(B1.max(initial=-1), A2.max(initial=-1)) + 1)
    if y is None:
        y = torch.empty(x.shape, dtype=torch.float32 if prec == "bf16" else x.dtype, device=x.device)
    for t in (Lenv, Renv, x, y):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("operands must be contiguous device tensors")
    torch.cuda.synchronize()
    I32 = C.POINTER(C.c_int32)
    DP = C.POINTER(C.c_double)
    rc = ctx.lib.tt_heff_apply_dev(ctx.h, PREC[prec], rl, rr, RA, RB, RC, C.c_void_p(Lenv.data_ptr()),
                                   C.c_void_p(Renv.data_ptr()), len(A1), A1.ctypes.data_as(I32),
                                   B1.ctypes.data_as(I32), o1.ctypes.data_as(DP), len(A2), A2.ctypes.data_as(I32),
                                   B2.ctypes.data_as(I32), o2.ctypes.data_as(DP), C.c_void_p(x.data_ptr()),
                                   C.c_void_p(y.data_ptr()))
    ctx._check(rc)
    return y


def heff_apply_rb(ctx, prec, Lenv, W1, W2, Renv, x, RB, y=None):
    """As heff_apply with an explicit middle channel count RB."""
    import torch

    RA, rl, _ = Lenv.shape
    RC, rr, _ = Renv.shape
    A1, B1, o1 = _sparse(W1)
    A2, B2, o2 = _sparse(W2)
    if y is None:
        y = torch.empty(x.shape, dtype=torch.float32 if prec == "bf16" else x.dtype, device=x.device)
    torch.cuda.synchronize()
    I32 = C.POINTER(C.c_int32)
    DP = C.POINTER(C.c_double)
    rc = ctx.lib.tt_heff_apply_dev(ctx.h, PREC[prec], rl, rr, RA, RB, RC, C.c_void_p(Lenv.data_ptr()),
                                   C.c_void_p(Renv.data_ptr()), len(A1), A1.ctypes.data_as(I32),
                                   B1.ctypes.data_as(I32), o1.ctypes.data_as(DP), len(A2), A2.ctypes.data_as(I32),
                                   B2.ctypes.data_as(I32), o2.ctypes.data_as(DP), C.c_void_p(x.data_ptr()),
                                   C.c_void_p(y.data_ptr()))
    ctx._check(rc)
    return y


def window_apply(ctx, b, ql, qr, Lenv, Renv, x, prec="f64", y=None):
    """y = H_eff x of the context's MPO at sites (b, b+1) with the given FP64
    device environments and bond labels (tt_window_apply_dev)."""
    import torch

    ql = np.ascontiguousarray(ql, dtype=np.int32)
    qr = np.ascontiguousarray(qr, dtype=np.int32)
    if y is None:
        y = torch.empty_like(x)
    torch.cuda.synchronize()
    I32 = C.POINTER(C.c_int32)
    rc = ctx.lib.tt_window_apply_dev(ctx.h, int(b), len(ql), len(qr), ql.ctypes.data_as(I32), qr.ctypes.data_as(I32),
                                     C.c_void_p(Lenv.data_ptr()), C.c_void_p(Renv.data_ptr()), PREC[prec],
                                     C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
    ctx._check(rc)
    return y


def gemm(ctx, prec, M, N, K, batch, kin, strides, a_kcontig, b_ncontig, A, B, Cout, alpha=1.0, beta=0.0):
    """Strided batched MFMA GEMM on device tensors (see tt_gemm_dev)."""
    import torch

    st = (C.c_longlong * 10)(*[int(s) for s in strides])
    torch.cuda.synchronize()
    rc = ctx.lib.tt_gemm_dev(ctx.h, PREC[prec], M, N, K, batch, kin, st, int(a_kcontig), int(b_ncontig), alpha, beta,
                             C.c_void_p(A.data_ptr()), C.c_void_p(B.data_ptr()), C.c_void_p(Cout.data_ptr()))
    ctx._check(rc)
    return Cout


def env_update(ctx, side, Env, Ubra, Uket, W, RA, RB, out=None):
    """One environment update (FP64 device tensors).  side 0: left, 1: right."""
    import torch

    A, B, o = _sparse(W)
    rb, rk = Ubra.shape[0], Uket.shape[0]
    rb2, rk2 = Ubra.shape[2], Uket.shape[2]
    if out is None:
        shape = (RB, rb2, rk2) if side == 0 else (RA, rb, rk)
        out = torch.empty(shape, dtype=torch.float64, device=Env.device)
    torch.cuda.synchronize()
    I32 = C.POINTER(C.c_int32)
    rc = ctx.lib.tt_env_update_dev(ctx.h, side, rb, rk, rb2, rk2, RA, RB, C.c_void_p(Env.data_ptr()),
                                   C.c_void_p(Ubra.data_ptr()), C.c_void_p(Uket.data_ptr()), len(A),
                                   A.ctypes.data_as(I32), B.ctypes.data_as(I32),
                                   o.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(out.data_ptr()))
    ctx._check(rc)
    return out


def heff_energy_grad(ctx, Lenv, W1, W2, Renv, x, RB):
    """E = <x|H_eff|x> and its gradients (FP64 device tensors; entry gradients on the host)."""
    import torch

    RA, rl, _ = Lenv.shape
    RC, rr, _ = Renv.shape
    A1, B1, o1 = _sparse(W1)
    A2, B2, o2 = _sparse(W2)
    gx = torch.empty_like(x)
    gL = torch.empty_like(Lenv)
    gR = torch.empty_like(Renv)
    g1 = np.zeros(16 * len(A1))
    g2 = np.zeros(16 * len(A2))
    E = C.c_double()
    torch.cuda.synchronize()
    I32 = C.POINTER(C.c_int32)
    DP = C.POINTER(C.c_double)
    rc = ctx.lib.tt_heff_energy_grad_dev(ctx.h, rl, rr, RA, RB, RC, C.c_void_p(Lenv.data_ptr()),
                                         C.c_void_p(Renv.data_ptr()), len(A1), A1.ctypes.data_as(I32),
                                         B1.ctypes.data_as(I32), o1.ctypes.data_as(DP), len(A2),
                                         A2.ctypes.data_as(I32), B2.ctypes.data_as(I32), o2.ctypes.data_as(DP),
                                         C.c_void_p(x.data_ptr()), C.byref(E), C.c_void_p(gx.data_ptr()),
                                         C.c_void_p(gL.data_ptr()), C.c_void_p(gR.data_ptr()),
                                         g1.ctypes.data_as(DP), g2.ctypes.data_as(DP))
    ctx._check(rc)
    return E.value, gx, gL, gR, g1.reshape(-1, 4, 4), g2.reshape(-1, 4, 4)


def make_heff_energy(ctx, W1idx, W2idx, RB):
    """torch.autograd.Function for E = <x|H_eff|x> with the hand-written backward.

    ``W1idx``/``W2idx`` are (A, B) index arrays of the sparse cores; the local
    operators are differentiable inputs of shape [nnz, 4, 4]."""
    import torch

    class HeffEnergy(torch.autograd.Function):
        @staticmethod
        def forward(fctx, x, Lenv, Renv, ops1, ops2):
            E, gx, gL, gR, g1, g2 = heff_energy_grad(ctx, Lenv.detach(), (W1idx[0], W1idx[1], ops1.detach().cpu().numpy()),
                                                     (W2idx[0], W2idx[1], ops2.detach().cpu().numpy()), Renv.detach(),
                                                     x.detach(), RB)
            fctx.save_for_backward(gx, gL, gR, torch.from_numpy(g1), torch.from_numpy(g2))
            return torch.tensor(E, dtype=torch.float64)

        @staticmethod
        def backward(fctx, gE):
            gx, gL, gR, g1, g2 = fctx.saved_tensors
            s = gE.item()
            return s * gx, s * gL, s * gR, s * g1, s * g2

    return HeffEnergy
