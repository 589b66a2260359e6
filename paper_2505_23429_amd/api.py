"""Python binding with the names of the C ABI (include/tt.h).

Argument marshalling only: every step of the additive two-level DMRG path runs
in the HIP library.  PyTorch supplies device memory for the kernel-level entry
points; the context owns its own device state.
"""
from __future__ import annotations

import copy
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
                 sub_workers=0, mix_stage=0, svd_lds=True, worker_alloc_limit=0, stream=None, torch_alloc=False,
                 coarse_k=1, one_site=False, functional="eig", coarse_krylov=False,
                 graph_products=False, precontract=2, svd_blocked=1):
        """``stream``: a torch.cuda.Stream (or raw stream handle) every call runs on;
        ``torch_alloc``: take every device block of the context from the torch caching
        allocator (tt_opts.dev_alloc/dev_free) instead of the library's own pools;
        ``one_site``: one-site micro-steps (FP64 products) instead of two-site ones;
        ``functional``: "eig" (Rayleigh quotient, the eigenvalue problem) or "linear"
        (1/2 <X,AX> - <F,X> with F from ``set_rhs``; A must be positive definite);
        ``coarse_krylov``: Step 3 by Lanczos without forming the coarse matrix;
        ``graph_products``: replay the block-sparse products from HIP graphs;
        ``precontract``: 2 = contract each environment with its site's MPO tensor once
        per window (every product is then two GEMMs), 1 = only the left one, 0 = none
        (every product forms L x and applies both site tensors as sparse mixes);
        ``svd_blocked``: 1 = sector SVD blocks of 48 or more columns by the blocked Jacobi
        kernels (many workgroups per block), 0 = never, 2 = every block they take, 3 and 4 =
        as 2 with the pair kernels' rows per lane pinned to 0 (loops) or 9 (for testing)."""
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
        o.coarse_k = int(coarse_k)
        self.coarse_k = int(coarse_k)
        o.one_site = int(bool(one_site))
        if functional not in ("eig", "linear"):
            raise ValueError("functional must be 'eig' or 'linear'")
        o.functional = 1 if functional == "linear" else 0
        o.coarse_krylov = int(bool(coarse_krylov))
        o.graph_products = int(bool(graph_products))
        if precontract not in (0, 1, 2):
            raise ValueError("precontract must be 0, 1 or 2")
        o.precontract = int(precontract)
        if svd_blocked not in (0, 1, 2, 3, 4):
            raise ValueError("svd_blocked must be 0, 1, 2, 3 or 4")
        o.svd_blocked = int(svd_blocked)
        self.functional = functional
        if stream is not None:
            o.stream = C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        self._callbacks = None
        if torch_alloc:
            self._callbacks = _torch_allocator(device)
            o.dev_alloc = C.cast(self._callbacks[0], C.c_void_p)
            o.dev_free = C.cast(self._callbacks[1], C.c_void_p)
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

    def set_rhs(self, cores, labels):
        """Right-hand side F of the linear-system functional, as a TT (kept as given)."""
        Lsites = len(cores)
        r, rp = _iarr([c.shape[0] for c in cores] + [cores[-1].shape[2]])
        F, kf = _ptr_array([c.reshape(-1) for c in cores], C.c_double)
        q, kq = _ptr_array([np.asarray(l).reshape(-1) for l in labels], C.c_int32)
        self._check(self.lib.tt_set_rhs(self.h, Lsites, rp, F, q))

    def functional_value(self):
        """J(X) of the current iterate for the context's functional."""
        j = C.c_double()
        self._check(self.lib.tt_functional(self.h, C.byref(j)))
        return j.value

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
        """Steps 3-4 after local_solve over nsub subdomains (nsub * coarse_k + 1 coarse states)."""
        n = nsub * self.coarse_k + 1
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
        m = rep.nstates
        S = np.array(rep.S[: m * m]).reshape(m, m)
        A = np.array(rep.A[: m * m]).reshape(m, m)
        return {
            "status": rc, "E_before": rep.E_before, "E_local": np.array(rep.E_local[:n]),
            "matvecs": np.array(rep.matvecs[:n]), "matvecs_f64": np.array(rep.matvecs_f64[:n]),
            "S": S, "A": A, "c": np.array(rep.coef[:m]),
            "lambda": rep.lambda_, "rankS": rep.rankS, "E_after": rep.E_after, "discarded": rep.discarded,
            "seconds": list(rep.seconds), "flops_heff": rep.flops_heff, "seconds_heff": rep.seconds_heff,
            "phase_seconds": list(rep.phase_seconds), "b": np.array(rep.rhs[:m]),
            "coarse_matvecs": rep.coarse_matvecs,
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
    # the same timing slots as filled by two-site products with the precontracted left
    # operator (its GEMM takes the place of stage 1 and the first mix), with both
    # precontracted operators, and by one-site products (unused slots: "-")
    KERNELS_LEFT_OPERATOR = ("gemm_LWx", "-", "-", "-", "mix2_gather", "mix2_heavy_gemm", "mix2_heavy_scatter",
                             "gemm_R", "gemm_R_reduce")
    KERNELS_PRECONTRACTED = ("gemm_LWx_panels", "-", "-", "-", "-", "-", "-", "gemm_panels_WR", "gemm_panels_WR_reduce")
    KERNELS_ONE_SITE = ("env_s1_Lx", "env_mix_gather", "env_mix_heavy_gemm", "env_mix_heavy", "-", "-", "-",
                        "gemm_R_stacked", "gemm_R_stacked_reduce")

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


def _torch_allocator(device):
    """ctypes callbacks that hand out and take back blocks of the torch caching
    allocator (stream-ordered on the stream the library passes)."""
    import torch

    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(stream or 0))
        except RuntimeError:  # out of memory: the library reports TT_ENOMEM
            return None

    def free(ptr, stream, user):
        torch.cuda.caching_allocator_delete(int(ptr))

    return L.ALLOC_FN(alloc), L.FREE_FN(free)


def open_context(mpo, cores, labels, **kw):
    ctx = Context(**kw)
    ctx.set_mpo(mpo)
    ctx._L = mpo.L
    ctx.set_mps(cores, labels)
    return ctx


# ---- kernel-level entry points (device tensors from torch) -------------------
#
# Every device operand is validated before its pointer crosses the ABI: the
# library trusts the sizes implied by the other arguments, so a tensor of the
# wrong shape, dtype or layout would be read or written out of bounds.  Shape
# and dtype are checked before the device, so these errors are raised (as
# ValueError) without touching a GPU.

_DT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16"}


def _need(*specs):
    """Each spec is (tensor, name, dtype, shape or None, element count or None).
    Shapes, sizes, dtypes and layouts of all operands are checked first, then
    that every operand is a device tensor."""
    import torch

    for t, name, dtype, shape, numel in specs:
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
        if shape is not None and tuple(t.shape) != tuple(int(v) for v in shape):
            raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(int(v) for v in shape)}")
        if numel is not None and t.numel() < numel:
            raise ValueError(f"{name}: {t.numel()} elements, the call addresses {numel}")
        want = getattr(torch, dtype)
        if t.dtype != want:
            raise ValueError(f"{name}: dtype {t.dtype}, expected {want}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: must be contiguous")
    for t, name, *_ in specs:
        if not t.is_cuda:
            raise ValueError(f"{name}: must be a device tensor")


def _need_prec(prec):
    if prec not in PREC:
        raise ValueError(f"unknown precision {prec!r} (one of {sorted(PREC)})")


def _need_pad(name, v):
    if v <= 0 or v % 32:
        raise ValueError(f"{name} = {v} must be a positive multiple of 32")


def _sparse(W, R_in, R_out, name):
    A, B, ops = W
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    ops = np.ascontiguousarray(ops, dtype=np.float64)
    if A.ndim != 1 or A.shape != B.shape or ops.shape != (len(A), 4, 4):
        raise ValueError(f"{name}: entries (A[nnz], B[nnz], ops[nnz, 4, 4]) expected")
    if len(A) and (A.min() < 0 or A.max() >= R_in or B.min() < 0 or B.max() >= R_out):
        raise ValueError(f"{name}: channel index outside [0, {R_in}) x [0, {R_out})")
    return A, B, ops.reshape(-1)


def _pointers(*ts):
    return [C.c_void_p(t.data_ptr()) for t in ts]


def heff_apply_rb(ctx, prec, Lenv, W1, W2, Renv, x, RB, y=None):
    """y = H_eff x (tt_heff_apply_dev): device tensors Lenv [RA][rl][rl],
    Renv [RC][rr][rr], x [rl][4][4][rr] in the precision's element type (bf16:
    bfloat16 operands, float32 y), rl and rr multiples of 32; sparse cores
    W1 (RA -> RB), W2 (RB -> RC) on the host."""
    import torch

    _need_prec(prec)
    RA, rl, RC, rr = Lenv.shape[0], Lenv.shape[1], Renv.shape[0], Renv.shape[1]
    _need_pad("rl", rl)
    _need_pad("rr", rr)
    A1, B1, o1 = _sparse(W1, RA, RB, "W1")
    A2, B2, o2 = _sparse(W2, RB, RC, "W2")
    ydt = "float32" if prec == "bf16" else _DT[prec]
    ops = [(Lenv, "Lenv", _DT[prec], (RA, rl, rl), None), (Renv, "Renv", _DT[prec], (RC, rr, rr), None),
           (x, "x", _DT[prec], (rl, 4, 4, rr), None)]
    _need(*ops)
    if y is None:
        y = torch.empty(x.shape, dtype=getattr(torch, ydt), device=x.device)
    _need(*ops, (y, "y", ydt, (rl, 4, 4, rr), None))
    torch.cuda.synchronize()
    I32 = C.POINTER(C.c_int32)
    DP = C.POINTER(C.c_double)
    pL, pR, px, py = _pointers(Lenv, Renv, x, y)
    rc = ctx.lib.tt_heff_apply_dev(ctx.h, PREC[prec], rl, rr, RA, RB, RC, pL, pR, len(A1), A1.ctypes.data_as(I32),
                                   B1.ctypes.data_as(I32), o1.ctypes.data_as(DP), len(A2), A2.ctypes.data_as(I32),
                                   B2.ctypes.data_as(I32), o2.ctypes.data_as(DP), px, py)
    ctx._check(rc)
    return y


def heff_apply_noalloc(ctx, prec, Lenv, W1, W2, Renv, x, RB, y):
    """tt_heff_apply_dev_noalloc: heff_apply_rb ("f64" or "f32") without device
    allocation; the output y is the caller's.  Intermediates live in the library's
    fixed per-GPU scratch, so concurrent calls on one GPU must be serialised."""
    import torch

    if prec not in ("f64", "f32"):
        raise ValueError("heff_apply_noalloc: precision must be 'f64' or 'f32'")
    RA, rl, RC, rr = Lenv.shape[0], Lenv.shape[1], Renv.shape[0], Renv.shape[1]
    _need_pad("rl", rl)
    _need_pad("rr", rr)
    A1, B1, o1 = _sparse(W1, RA, RB, "W1")
    A2, B2, o2 = _sparse(W2, RB, RC, "W2")
    dt = _DT[prec]
    _need((Lenv, "Lenv", dt, (RA, rl, rl), None), (Renv, "Renv", dt, (RC, rr, rr), None),
          (x, "x", dt, (rl, 4, 4, rr), None), (y, "y", dt, (rl, 4, 4, rr), None))
    torch.cuda.synchronize()
    I32 = C.POINTER(C.c_int32)
    DP = C.POINTER(C.c_double)
    pL, pR, px, py = _pointers(Lenv, Renv, x, y)
    rc = ctx.lib.tt_heff_apply_dev_noalloc(ctx.h, PREC[prec], rl, rr, RA, RB, RC, pL, pR, len(A1),
                                           A1.ctypes.data_as(I32), B1.ctypes.data_as(I32), o1.ctypes.data_as(DP),
                                           len(A2), A2.ctypes.data_as(I32), B2.ctypes.data_as(I32),
                                           o2.ctypes.data_as(DP), px, py)
    ctx._check(rc)
    return y


def heff_apply(ctx, prec, Lenv, W1, W2, Renv, x, y=None):
    """As heff_apply_rb with RB = the largest middle channel index + 1."""
    RB = int(max(np.max(W1[1], initial=-1), np.max(W2[0], initial=-1)) + 1)
    return heff_apply_rb(ctx, prec, Lenv, W1, W2, Renv, x, RB, y)


def window_apply(ctx, b, ql, qr, Lenv, Renv, x, prec="f64", y=None):
    """y = H_eff x of the context's MPO at sites (b, b+1) with FP64 device
    environments Lenv [R_b][rlp][rlp], Renv [R_{b+2}][rrp][rrp] and x
    [rlp][4][4][rrp] (rlp, rrp: bond dimensions padded to 32), bond labels on
    the host (tt_window_apply_dev)."""
    import torch

    _need_prec(prec)
    ql = np.ascontiguousarray(ql, dtype=np.int32)
    qr = np.ascontiguousarray(qr, dtype=np.int32)
    if ql.ndim != 2 or ql.shape[1] != 2 or qr.ndim != 2 or qr.shape[1] != 2:
        raise ValueError("ql, qr: (N, 2Sz) label arrays of shape [r][2] expected")
    rlp, rrp = -(-len(ql) // 32) * 32, -(-len(qr) // 32) * 32
    if Lenv.ndim != 3 or Renv.ndim != 3:
        raise ValueError("Lenv, Renv: [channels][bra][ket] expected")
    ops = [(Lenv, "Lenv", "float64", (Lenv.shape[0], rlp, rlp), None),
           (Renv, "Renv", "float64", (Renv.shape[0], rrp, rrp), None), (x, "x", "float64", (rlp, 4, 4, rrp), None)]
    _need(*ops)
    if y is None:
        y = torch.empty_like(x)
    _need(*ops, (y, "y", "float64", (rlp, 4, 4, rrp), None))
    torch.cuda.synchronize()
    I32 = C.POINTER(C.c_int32)
    pL, pR, px, py = _pointers(Lenv, Renv, x, y)
    rc = ctx.lib.tt_window_apply_dev(ctx.h, int(b), len(ql), len(qr), ql.ctypes.data_as(I32), qr.ctypes.data_as(I32),
                                     pL, pR, PREC[prec], px, py)
    ctx._check(rc)
    return y


def gemm(ctx, prec, M, N, K, batch, kin, strides, a_kcontig, b_ncontig, A, B, Cout, alpha=1.0, beta=0.0):
    """Strided batched MFMA GEMM on device tensors (see tt_gemm_dev).  Every
    operand must hold the largest element offset its strides address."""
    import torch

    _need_prec(prec)
    st = [int(s) for s in strides]
    if len(st) != 10 or min(st) < 0:
        raise ValueError("strides: ten non-negative element strides expected")
    if min(M, N, K, batch) < 0 or kin <= 0 or K % kin:
        raise ValueError("sizes: M, N, K, batch >= 0 and K a multiple of kin expected")
    sAb, sAm, sAkb, sAkk, sBb, sBkb, sBkk, sBn, sCb, sCm = st
    if M * N * batch > 0:
        kb = K // kin
        last_a = (batch - 1) * sAb + (M - 1) * sAm + max(kb - 1, 0) * sAkb + (kin - 1) * sAkk if K else -1
        last_b = (batch - 1) * sBb + max(kb - 1, 0) * sBkb + (kin - 1) * sBkk + (N - 1) * sBn if K else -1
        last_c = (batch - 1) * sCb + (M - 1) * sCm + (N - 1)
        cdt = "float32" if prec == "bf16" else _DT[prec]
        _need((A, "A", _DT[prec], None, last_a + 1), (B, "B", _DT[prec], None, last_b + 1),
              (Cout, "C", cdt, None, last_c + 1))
    st = (C.c_longlong * 10)(*st)
    torch.cuda.synchronize()
    pa, pb, pc = _pointers(A, B, Cout)
    rc = ctx.lib.tt_gemm_dev(ctx.h, PREC[prec], M, N, K, batch, kin, st, int(a_kcontig), int(b_ncontig), alpha, beta,
                             pa, pb, pc)
    ctx._check(rc)
    return Cout


def env_update(ctx, side, Env, Ubra, Uket, W, RA, RB, out=None):
    """One environment update (FP64 device tensors; bond dimensions multiples of
    32).  side 0: left, Env [RA][rb][rk] -> out [RB][rb2][rk2]; side 1: right,
    Env [RB][rb2][rk2] -> out [RA][rb][rk]."""
    import torch

    if side not in (0, 1):
        raise ValueError("side must be 0 (left) or 1 (right)")
    A, B, o = _sparse(W, RA, RB, "W")
    if Ubra.ndim != 3 or Uket.ndim != 3:
        raise ValueError("Ubra, Uket: cores [r][4][r'] expected")
    rb, rk = Ubra.shape[0], Uket.shape[0]
    rb2, rk2 = Ubra.shape[2], Uket.shape[2]
    for nm, v in (("rb", rb), ("rk", rk), ("rb2", rb2), ("rk2", rk2)):
        _need_pad(nm, v)
    ein, eout = ((RA, rb, rk), (RB, rb2, rk2)) if side == 0 else ((RB, rb2, rk2), (RA, rb, rk))
    ops = [(Ubra, "Ubra", "float64", (rb, 4, rb2), None), (Uket, "Uket", "float64", (rk, 4, rk2), None),
           (Env, "Env", "float64", ein, None)]
    _need(*ops)
    if out is None:
        out = torch.empty(eout, dtype=torch.float64, device=Env.device)
    _need(*ops, (out, "out", "float64", eout, None))
    torch.cuda.synchronize()
    I32 = C.POINTER(C.c_int32)
    pE, pb, pk, po = _pointers(Env, Ubra, Uket, out)
    rc = ctx.lib.tt_env_update_dev(ctx.h, side, rb, rk, rb2, rk2, RA, RB, pE, pb, pk, len(A), A.ctypes.data_as(I32),
                                   B.ctypes.data_as(I32), o.ctypes.data_as(C.POINTER(C.c_double)), po)
    ctx._check(rc)
    return out


def heff_energy_grad(ctx, Lenv, W1, W2, Renv, x, RB):
    """E = <x|H_eff|x> and its gradients (tt_heff_energy_grad_dev): FP64 device
    tensors Lenv [RA][rl][rl], Renv [RC][rr][rr], x [rl][4][4][rr] (rl, rr
    multiples of 32); returns E, gx, gL, gR on the device and the per-entry
    operator gradients of W1 and W2 on the host."""
    import torch

    RA, rl, RC, rr = Lenv.shape[0], Lenv.shape[1], Renv.shape[0], Renv.shape[1]
    _need_pad("rl", rl)
    _need_pad("rr", rr)
    A1, B1, o1 = _sparse(W1, RA, RB, "W1")
    A2, B2, o2 = _sparse(W2, RB, RC, "W2")
    _need((Lenv, "Lenv", "float64", (RA, rl, rl), None), (Renv, "Renv", "float64", (RC, rr, rr), None),
          (x, "x", "float64", (rl, 4, 4, rr), None))
    gx = torch.empty_like(x)
    gL = torch.empty_like(Lenv)
    gR = torch.empty_like(Renv)
    g1 = np.zeros(16 * len(A1))
    g2 = np.zeros(16 * len(A2))
    E = C.c_double()
    torch.cuda.synchronize()
    I32 = C.POINTER(C.c_int32)
    DP = C.POINTER(C.c_double)
    pL, pR, px, pgx, pgL, pgR = _pointers(Lenv, Renv, x, gx, gL, gR)
    rc = ctx.lib.tt_heff_energy_grad_dev(ctx.h, rl, rr, RA, RB, RC, pL, pR, len(A1), A1.ctypes.data_as(I32),
                                         B1.ctypes.data_as(I32), o1.ctypes.data_as(DP), len(A2),
                                         A2.ctypes.data_as(I32), B2.ctypes.data_as(I32), o2.ctypes.data_as(DP), px,
                                         C.byref(E), pgx, pgL, pgR, g1.ctypes.data_as(DP), g2.ctypes.data_as(DP))
    ctx._check(rc)
    return E.value, gx, gL, gR, g1.reshape(-1, 4, 4), g2.reshape(-1, 4, 4)


def make_heff_energy(ctx, W1idx, W2idx, RB):
    """torch.autograd.Function for E = <x|H_eff|x> whose backward is the
    library's hand-written one (tt_heff_energy_grad_dev).

    ``W1idx``/``W2idx`` are the (A, B) index arrays of the two sparse cores; the
    local operators are differentiable inputs ``ops1``/``ops2`` of shape
    [nnz, 4, 4] (host or device).  ``apply(x, Lenv, Renv, ops1, ops2)`` returns
    E as a 0-d float64 tensor on x's device; every gradient comes back on its
    input's device in its input's dtype."""
    import torch

    class HeffEnergy(torch.autograd.Function):
        @staticmethod
        def forward(fctx, x, Lenv, Renv, ops1, ops2):
            E, gx, gL, gR, g1, g2 = heff_energy_grad(
                ctx, Lenv.detach(), (W1idx[0], W1idx[1], ops1.detach().cpu().numpy()),
                (W2idx[0], W2idx[1], ops2.detach().cpu().numpy()), Renv.detach(), x.detach(), RB)
            g1 = torch.from_numpy(g1).to(device=ops1.device, dtype=ops1.dtype)
            g2 = torch.from_numpy(g2).to(device=ops2.device, dtype=ops2.dtype)
            fctx.save_for_backward(gx, gL, gR, g1, g2)
            return torch.tensor(E, dtype=torch.float64, device=x.device)

        @staticmethod
        def backward(fctx, gE):
            gx, gL, gR, g1, g2 = fctx.saved_tensors
            return gE * gx, gE * gL, gE * gR, gE.to(g1.device) * g1, gE.to(g2.device) * g2

    return HeffEnergy


def make_mpo_energy(ctx, mpo):
    """torch.autograd.Function for E(ops) = <U|H(ops)|U> of the context's current
    (normalised) iterate, where ``ops`` [sum_k nnz_k, 4, 4] are the local operators
    of every MPO entry (sites in order, the entry structure of ``mpo``).  Forward:
    the environment chain (tt_energy, after tt_set_mpo with these operators when
    they differ from the context's).  Backward: the library's hand-written
    backward through the environment chains (tt_energy_mpo_grad, environments
    recomputed).  Composed with ``mpo_linear_map`` it gives dE/dh by autograd."""
    import torch

    nnz = [len(a) for a in mpo.A]
    offs = np.concatenate([[0], np.cumsum(nnz)])
    state = {"ops": np.concatenate([o.reshape(-1, 4, 4) for o in mpo.ops], axis=0)}

    def _set(ops_np):
        if ops_np.shape != state["ops"].shape:
            raise ValueError(f"ops: shape {ops_np.shape}, expected {state['ops'].shape}")
        if not np.array_equal(ops_np, state["ops"]):
            m2 = copy.copy(mpo)
            m2.ops = [ops_np[offs[k]:offs[k + 1]] for k in range(mpo.L)]
            ctx.set_mpo(m2)
            state["ops"] = ops_np.copy()

    class MpoEnergy(torch.autograd.Function):
        @staticmethod
        def forward(fctx, ops):
            _set(np.ascontiguousarray(ops.detach().cpu().numpy(), dtype=np.float64))
            fctx.dev, fctx.dt = ops.device, ops.dtype
            return torch.tensor(ctx.energy(), dtype=torch.float64, device=ops.device)

        @staticmethod
        def backward(fctx, gE):
            _, gops = ctx.mpo_gradient(mpo)
            g = torch.from_numpy(np.concatenate(gops, axis=0)).to(device=fctx.dev, dtype=fctx.dt)
            return gE.to(g.device) * g

    return MpoEnergy


def mpo_linear_map(mpo, h0):
    """The local operators of every MPO entry as a differentiable function of
    the one-body integrals: ops(h) = ops(h0) + sum_pq (h - h0)_pq D_pq, exact
    because every entry is linear in h (D from the builder's derivative map)."""
    import torch

    L = mpo.L
    nnz = [len(a) for a in mpo.A]
    offs = np.concatenate([[0], np.cumsum(nnz)])
    base = torch.from_numpy(np.concatenate([o.reshape(-1, 4, 4) for o in mpo.ops], axis=0))
    rows = torch.tensor([offs[k] + e for k, e, _, _, _ in mpo.dh], dtype=torch.long)
    pq = torch.tensor([p * L + q for _, _, p, q, _ in mpo.dh], dtype=torch.long)
    D = torch.from_numpy(np.stack([np.asarray(d).reshape(4, 4) for *_, d in mpo.dh]))
    h0 = torch.as_tensor(np.asarray(h0, dtype=np.float64))

    def ops_of(h):
        dh = (h - h0).reshape(-1)[pq]
        return base.index_add(0, rows, dh[:, None, None] * D)

    return ops_of
