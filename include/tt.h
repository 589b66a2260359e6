/*
 * tt.h — C ABI of the additive two-level DMRG hot path on one AMD MI355X (gfx950).
 *
 * The library computes, for a Hamiltonian given as a matrix product operator
 * (eq. MPO, Appendix A) and a tensor-train iterate (Definitions "tensor train
 * parameter space" and "tensor train contraction mapping", Section 2.1):
 *   - the two-site effective-Hamiltonian product (the two-site form of
 *     eq. mat_vec built from the environments eq. env_L / eq. env_R),
 *   - the local eigenproblems of the two-site micro-iteration
 *     (eq. MALS_Micro, Lemma "DMRG micro-iterations for eigenvalue problems"),
 *     run over groups of adjoining sites (Extension Two of Algorithm 2),
 *   - the coarse-space minimisation (eq. d_optim, eq. d_opt_lin_3/4,
 *     eq. A_reduced, rank-deficient branch eq. aux_eig_final_sym) and the
 *     compression back to a left-orthogonal TT (Step 4 of Algorithm 2),
 *   - one global iteration of Algorithm 2 (two-site branch),
 *   - the classical two-site sweep (Algorithm 1, two-site branch).
 *
 * Conventions
 *   sites k = 0..L-1, local dimension 4 (|0>,|up>,|dn>,|updn>), bonds 0..L.
 *   TT core k:  U[a][s][b], row-major, a < r_k, b < r_{k+1}, r_0 = r_L = 1.
 *   MPO core k: W[A][s_out][s_in][B], given sparsely as nnz entries
 *               (A, B, op[4][4]) with op row-major [s_out][s_in].
 *   Environments: E[K][bra][ket] (operator channel outermost).
 *   Quantum-number labels are (N, 2Sz) int32 pairs.
 *   Two-site tensor: x[a][s1][s2][b].
 *
 * Ownership: host arrays are read during the call and copied; the caller keeps
 * them.  Device pointers passed to the *_dev entry points are borrowed for the
 * duration of the call and used on the context's stream (tt_opts.stream, or
 * the context's own; the call returns after the stream is synchronised).  The
 * context holds all other device memory it needs: from the caller's allocator
 * callbacks (tt_opts.dev_alloc/dev_free) when given, otherwise from its own
 * pools of hipMalloc'ed chunks on the context's device; tt_destroy releases it.
 *
 * Errors: no exception crosses the ABI.  Return value 0 = success, > 0 =
 * warning (result usable), < 0 = error; tt_last_error() gives a message.
 * Sizes and quantum-number structure are validated on the host before any
 * device work.
 */
#ifndef TT_H
#define TT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_OK 0
#define TT_WNOCONV 1      /* a local or coarse eigensolve hit its iteration limit */
#define TT_WRANKDEF 2     /* the coarse overlap matrix was rank-deficient (eps branch) */
#define TT_EINVAL (-1)    /* shape / quantum-number mismatch, bad argument */
#define TT_ESTATE (-2)    /* wrong call order */
#define TT_ENOMEM (-3)    /* device allocation failed */
#define TT_EHIP (-4)      /* HIP / rocSOLVER runtime error */
#define TT_EINTERNAL (-5) /* unexpected internal failure */

typedef enum { TT_F64 = 0, TT_F32 = 1, TT_BF16 = 2 } tt_prec;

typedef struct tt_opts {
  int chi_max;        /* maximal TT rank kept by every truncation */
  double svd_cutoff;  /* drop singular values below svd_cutoff * s_max (1e-12) */
  double tie_rel;     /* tie group |s_i - s_chi| <= tie_rel * s_max dropped if it straddles the cut */
  double dav_tol;     /* residual 2-norm tolerance of the local eigensolver (unit Ritz vector) */
  int dav_maxiter;    /* matvec limit per local eigensolve */
  int dav_maxsub;     /* subspace size before a restart */
  double coarse_eps;  /* keep overlap eigenvalues >= coarse_eps * max (rank-deficient branch) */
  int matvec_prec;    /* tt_prec of the effective-Hamiltonian product */
  int refine_fp64;    /* 1: after the low-precision phase, an FP64-anchored refinement to
                         dav_tol: residuals from FP64 products, correction directions from
                         low-precision ones (FP32; a bfloat16 solve continues in FP32) */
  double lowprec_tol; /* with refine_fp64: the low-precision phase ends when the residual is
                         <= lowprec_tol * |Ritz value| (or has stalled at the rounding floor
                         of the low-precision product); FP64 products then reach dav_tol */
  int device;         /* HIP device ordinal */
  int qn_skip;        /* 1: skip the exact zeros of the quantum-number blocks in the
                         effective-Hamiltonian product and environment updates */
  int sub_workers;    /* Step 2 (Algorithm 2): the subdomain solves are independent and run
                         concurrently on this many workers, each a host thread with its own
                         HIP stream, rocBLAS handle and workspaces; 0 = 4.  With 1 every
                         kernel is launched from the calling thread on the context's stream
                         (no worker threads).  If a worker's task runs out of device memory,
                         that task (and any not yet started) is run again one after another
                         on the context, and later calls use as many workers as fitted.
                         Results do not depend on it. */
  int mix_stage;      /* light rows of the block-sparse product's channel mixes: 0 = stage a
                         tile's distinct input rows in LDS where the group's operator entries
                         outnumber its distinct input rows 1.5 times or more, 1 = stage every
                         tile, 2 = never (read every entry's input directly).  Results do not
                         depend on it up to the rounding of FMA contraction. */
  int svd_lds;        /* sector SVDs: 1 = a charge block whose factors fit in LDS is factored
                         there, 0 = every block works in global memory (same arithmetic) */
  long long worker_alloc_limit; /* for testing the recovery from device memory exhaustion: a
                         task on a concurrent worker whose device allocations exceed this many
                         bytes fails as if the device were full (0 = no limit).  Such tasks,
                         like those of a real exhaustion, are run again one after another on
                         the context, with the same result. */
  void* stream;       /* hipStream_t of the caller (e.g. torch.cuda.current_stream), or NULL:
                         the context's own stream.  Every call of the context runs on it and
                         returns after it is synchronised.  Not destroyed by tt_destroy. */
  void* (*dev_alloc)(size_t bytes, void* stream, void* user);
                      /* caller's device allocator (e.g. the torch caching allocator), or NULL:
                         the library's own pools.  Called on the thread that needs the block,
                         with the stream the block will be used on; returns NULL when out of
                         memory (the call then fails with TT_ENOMEM or, on a concurrent worker,
                         recovers as for worker_alloc_limit).  Must be thread-safe. */
  void (*dev_free)(void* ptr, void* stream, void* user);
                      /* releases a block from dev_alloc (same stream argument); the library has
                         synchronised the stream before the call.  Set both callbacks or none.
                         Blocks live until the call that frees them or tt_destroy, so the
                         callbacks must stay valid until tt_destroy returns. */
  void* alloc_user;   /* passed to dev_alloc/dev_free */
  int coarse_k;       /* Extension One (Remark "Extensions of the A2DMRG algorithm"): the last
                         micro-step of every subdomain keeps its coarse_k lowest eigenvectors
                         (FP64 products), each giving an updated TT, so the coarse space has
                         nsub * coarse_k + 1 states (<= TT_MAX_SUB + 1); 1 = the plain method */
  int one_site;       /* 0: two-site micro-steps (Algorithm 2, two-site branch); 1: one-site
                         micro-steps (Algorithm 2, one-site branch, Definition "One-site and
                         two-site DMRG micro-iterations"): subdomain j optimises the cores of its
                         sites s_j..e_j one after another, moving the centre right by a
                         charge-block QR (the orthogonalization step of Algorithm 1), so bond
                         dimensions do not change in Step 2.  Needs matvec_prec = TT_F64 and
                         qn_skip = 1 (EINVAL otherwise). */
  int functional;     /* 0: J(X) = <X,AX>/<X,X> (eq. energy_eig, the eigenvalue problem);
                         1: J(X) = 1/2 <X,AX> - <F,X> (eq. energy_lin) with A the MPO operator,
                         which must be symmetric positive definite on the sector, and F the
                         TT given by tt_set_rhs.  The micro-steps then solve the projected
                         linear systems P^T A P w = P^T F (preconditioned conjugate gradients
                         to dav_tol relative to |P^T F|, at most dav_maxiter products) and
                         Step 3 the coarse linear system (Section "The second-level
                         minimization", last remark).  Needs matvec_prec = TT_F64, qn_skip = 1
                         and coarse_k = 1 (EINVAL otherwise). */
  int coarse_krylov;  /* 1: Step 3 without forming the coarse Hamiltonian matrix (Appendix on
                         the second-level problem, Krylov remark, eq. aux_mat-vec_prod): S is
                         formed, then the lowest eigenpair of the reduced problem comes from
                         Lanczos iterations whose products z_i = <U^i|H|W(v)> contract every
                         coarse state with the structured combination W(v) = sum_j v_j U^j (the
                         block TT of Step 4, bonds regrouped by charge) through one left and
                         one right environment chain and a branch per update.  The report's A
                         is then NaN.  functional = 0 only (EINVAL otherwise). */
  int graph_products; /* 1: each local problem's block-sparse two-site products replay a HIP
                         graph of their launches (captured at the second product; the first
                         runs eagerly), saving the per-kernel launch cost; results are bit for
                         bit those of eager launches.  Off while tt_kernel_timing records. */
  int precontract;    /* block-sparse two-site products (eq. mat_vec): which MPO site tensors are
                         contracted with their environment once per window instead of in every
                         product.  0 = none: every product forms L_A x for all left channels,
                         applies W1 and then W2 as sparse combinations of rows, and contracts
                         with R.  1 = the left operator LW[B] = sum_A W1[A, s1', s1, B] L_A
                         (formed in FP64): every product applies it to x in one grouped
                         matrix-core GEMM, then W2 and R as for 0.  2 (default) = the left and
                         the right operator WR[B] = sum_C W2[B, s2', s2, C] R_C: every product
                         is one GEMM with LW into panels of the bra's left half and one split-K
                         GEMM of the panels with WR; with matvec_prec = TT_BF16, LW, WR, x and
                         the panels are held in bfloat16 (FP32 arithmetic).  Same contraction,
                         different summation order. */
  int svd_blocked;    /* sector SVDs: 1 (default) = a block of at least 48 columns (and rows +
                         columns <= 1152) is factored by the blocked Jacobi kernels, spread
                         over many workgroups (two 8-column blocks of its columns per
                         workgroup); 0 = never; 2 = every block of 2 or more columns they take;
                         3 and 4 = as 2 with the rows per lane of their pair kernels pinned (0:
                         loops over LDS, 9: registers) instead of chosen by size (2-4 are for
                         testing).  Same rotations, visited in another order: results agree to
                         rounding. */
} tt_opts;

#define TT_MAX_SUB 64

typedef struct tt_sweep_report {
  int nsub;
  double E_before;                 /* <U|H|U> of the input iterate (functional 1: J(X)) */
  double E_local[TT_MAX_SUB];      /* last Ritz value of each subdomain sweep (functional 1: the
                                      local minimum 1/2 w.Aw - b.w of its last micro-step) */
  int matvecs[TT_MAX_SUB];         /* effective-Hamiltonian products per subdomain */
  double S[(TT_MAX_SUB + 1) * (TT_MAX_SUB + 1)]; /* coarse overlap, row-major (nsub+1)^2 */
  double A[(TT_MAX_SUB + 1) * (TT_MAX_SUB + 1)]; /* coarse Hamiltonian, row-major */
  double coef[TT_MAX_SUB + 1];     /* coarse coefficients: c^T S c = 1 (functional 0), the coarse
                                      minimiser (1); state 0 is the normalised iterate and every
                                      update is normalised, so S has a unit diagonal */
  double lambda;                   /* lowest coarse eigenvalue (functional 1: coarse minimum of J) */
  int rankS;                       /* numerical rank of S */
  double E_after;                  /* <U|H|U> of the compressed next iterate (functional 1: J) */
  double discarded;                /* total discarded weight of Step 4 */
  double seconds[4];               /* wall time of Steps 1..4 */
  double flops_heff;               /* dense-bond flops of all effective-Hamiltonian products */
  double seconds_heff;             /* device time of those products (HIP events) */
  double phase_seconds[9];         /* wall time: LQ sweep, step-1 environments, window set-up,
                                      Davidson, two-site splits, subdomain environment updates,
                                      coarse matrices, coarse solve + compression, all subdomain
                                      solves; with concurrent solves entries 2-5 are summed over
                                      the workers */
  int matvecs_f64[TT_MAX_SUB];     /* of matvecs[]: the products taken in FP64 */
  int nstates;                     /* coarse states n = nsub * coarse_k + 1: S, A are n x n, coef n */
  double rhs[TT_MAX_SUB + 1];      /* functional = 1: coarse right-hand side b_j = <F|U^j> */
  int coarse_matvecs;              /* coarse_krylov = 1: products with the coarse matrix */
} tt_sweep_report;

void tt_default_opts(tt_opts* o);
int tt_create(const tt_opts* opts, void** ctx_out);
void tt_destroy(void* ctx);
const char* tt_last_error(const void* ctx);

/* Operator A as an MPO (eq. MPO).  R[0..L] bond dimensions with R[0] = R[L] = 1;
 * per site k: nnz[k] entries A[k][e], B[k][e], ops[k][16*e..]; chan_q[k] holds
 * R[k] (dN, d2Sz) pairs (charge of the left operator of each channel).
 * block[4*k..4*k+3] = (p0, p1, q0, q1) marks an optional coefficient block of
 * site k: every entry with A in [p0,p1) and B in [q0,q1) must have an
 * identity local operator (times a coefficient); such blocks are applied as
 * dense channel transforms of the environments.  Use -1 for none. */
int tt_set_mpo(void* ctx, int L, const int* R, const int* nnz, const int32_t* const* A, const int32_t* const* B,
               const double* const* ops, const int32_t* const* chan_q, const int* block);

/* TT iterate (Definition "tensor train parameter space").  r[0..L], cores
 * U[k] host [r_k][4][r_{k+1}], labels q[k] host int32 [r_k][2].  Every core
 * must respect the labels (q(a) + q(s) = q(b)); the library brings the TT to
 * left-orthogonal form (sector-wise QR on the device) and normalises it. */
int tt_set_mps(void* ctx, int L, const int* r, const double* const* U, const int32_t* const* q);

/* Copy the current (left-orthogonal) iterate out.  If U is NULL only r[0..L] is
 * written; otherwise U[k] and q[k] must have room for the sizes in r.  With
 * functional = 1 the iterate keeps its norm (the last core carries it); with 0
 * it is normalised. */
int tt_get_mps(void* ctx, int* r, double* const* U, int32_t* const* q);

/* <U|H|U> / <U|U> of the current iterate. */
int tt_energy(void* ctx, double* E);

/* Right-hand side F of the linear-system functional (eq. energy_lin) as a TT:
 * r[0..L], cores F[k] host [r_k][4][r_{k+1}], labels q[k] host int32 [r_k][2]
 * (same conventions and checks as tt_set_mps; the cores are kept as given, not
 * orthogonalised or normalised).  Needs the MPO; F's sector must be the
 * iterate's (right boundary label), else the sweep fails with EINVAL. */
int tt_set_rhs(void* ctx, int L, const int* r, const double* const* F, const int32_t* const* q);

/* J(X) of the current iterate for the context's functional: the Rayleigh
 * quotient (functional 0) or 1/2 <X,AX> - <F,X> (functional 1). */
int tt_functional(void* ctx, double* J);

/* Keeps a device copy of the current iterate (op 0) or makes the kept copy the
 * current iterate again (op 1), without a host round trip: repeated global
 * iterations from one state.  TT_ESTATE if there is nothing to keep/restore
 * or the kept iterate does not fit the MPO; TT_EINVAL for another op. */
int tt_mps_checkpoint(void* ctx, int op);

/* Steps 1-2 of Algorithm 2: LQ sweep with saved orthogonal copies and
 * environment caches, then the local solves of nsub subdomains of lengths[]
 * sites (sum = L); subdomain j sweeps its bonds left to right, the last one
 * stopping at bond (L-2, L-1). */
int tt_local_solve(void* ctx, int nsub, const int* lengths, double* E_local, int* matvecs);

/* Steps 3-4: coarse matrices over {current, subdomain updates}, coarse
 * eigenpair, compression of the combination to chi_max; the result becomes
 * the current iterate.  S_out/A_out are row-major n x n and coef_out n long,
 * n = nsub * coarse_k + 1 (states ordered: current iterate, then per subdomain
 * its updates from the lowest local eigenvector up). */
int tt_coarse_correct(void* ctx, double* S_out, double* A_out, double* coef_out, double* lambda_out,
                      double* E_out, int* rankS_out);

/* One global iteration of Algorithm 2 (Steps 1-4). */
int tt_sweep(void* ctx, int nsub, const int* lengths, tt_sweep_report* out);

/* nsweeps full sweeps of classical two-site DMRG (Algorithm 1); energies[2*nsweeps]
 * receive the last Ritz value of every half sweep. */
int tt_dmrg2(void* ctx, int nsweeps, double* energies);

/* Kernel-level entry points (device pointers, borrowed).
 * Two-site product y = H_eff x with left environment Lenv[RA][rl][rl],
 * right environment Renv[RC][rr][rr], MPO cores W1 (RA -> RB) and W2 (RB -> RC)
 * given sparsely on the host, x, y [rl][4][4][rr].  Element type by prec:
 * TT_F64 double, TT_F32 float, TT_BF16 uint16 bfloat16 for Lenv/Renv/x with
 * float y.  rl and rr must be multiples of 32. */
int tt_heff_apply_dev(void* ctx, int prec, int rl, int rr, int RA, int RB, int RC, const void* Lenv,
                      const void* Renv, int nnz1, const int32_t* A1, const int32_t* B1, const double* ops1, int nnz2,
                      const int32_t* A2, const int32_t* B2, const double* ops2, const void* x, void* y);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tt_heff_apply_dev (TT_F64 or TT_F32)
 * without any device allocation.  Its intermediates (max(RA, RC) + RB slabs of
 * rl*16*rr elements) and the two cores' entry tables are carved from one fixed device
 * array of TT_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on holds
 * until the process ends; its address is looked up once per device by tt_create.  A
 * product that needs more scratch is refused with TT_EINVAL and a message naming the
 * size.  Every call on one GPU shares that GPU's array and overwrites it, so calls that
 * overlap in time on one GPU (two threads, or two contexts' streams) race: serialise
 * them.  Operands, layouts and results as tt_heff_apply_dev; the host entry tables are
 * copied with hipMemcpyAsync on the context's stream, and the call returns after the
 * stream is synchronised. */
#define TT_NOALLOC_SCRATCH_BYTES (256ull << 20)
int tt_heff_apply_dev_noalloc(void* ctx, int prec, int rl, int rr, int RA, int RB, int RC, const void* Lenv,
                              const void* Renv, int nnz1, const int32_t* A1, const int32_t* B1, const double* ops1,
                              int nnz2, const int32_t* A2, const int32_t* B2, const double* ops2, const void* x,
                              void* y);

/* Two-site product of the context's MPO at sites (b, b+1), y = H_eff x
 * (eq. mat_vec with the two-site contraction of Section 3), through the same
 * quantum-number block-sparse kernels the local solves use.  rl, rr: bond
 * dimensions at bonds b and b+2; ql [rl][2], qr [rr][2]: host (N, 2Sz) labels
 * of those bonds, equal labels contiguous (otherwise the dense product with
 * zero-block skipping is used).  Lenv: device FP64 [R_b][rlp][rlp] (bra, ket),
 * Renv: device FP64 [R_{b+2}][rrp][rrp], x, y: device FP64 [rlp][4][4][rrp],
 * with rlp, rrp = rl, rr rounded up to multiples of 32 (padding zero).
 * Entries of Lenv, Renv, x outside their charge blocks must be zero; prec
 * selects the arithmetic (TT_F64, TT_F32, or FP32 on bfloat16-rounded
 * operands for TT_BF16).  y is overwritten.  TT_EINVAL on bad arguments,
 * TT_ESTATE without an MPO. */
int tt_window_apply_dev(void* ctx, int b, int rl, int rr, const int32_t* ql, const int32_t* qr, const double* Lenv,
                        const double* Renv, int prec, const double* x, double* y);

/* One environment update (double precision).  side 0: left update
 * out[B][rb2][rk2] = sum E[A][rb][rk] Ubra[rb][4][rb2] W[A,s',s,B] Uket[rk][4][rk2];
 * side 1: right update out[A][rb][rk] = sum Ubra[rb][4][rb2] W Uket[rk][4][rk2] E[B][rb2][rk2].
 * RA/RB are the channel counts at the left/right bond of the site.  All bond
 * dimensions must be multiples of 32. */
int tt_env_update_dev(void* ctx, int side, int rb, int rk, int rb2, int rk2, int RA, int RB, const double* E,
                      const double* Ubra, const double* Uket, int nnz, const int32_t* A, const int32_t* B,
                      const double* ops, double* out);

/* Strided batched GEMM on MFMA (the building block of every contraction
 * above), C[b] = alpha * op(A[b]) op(B[b]) + beta * C[b] with
 * A(m,k) = A + b*sAb + m*sAm + (k/kin)*sAkb + (k%kin)*sAkk,
 * B(k,n) = B + b*sBb + (k/kin)*sBkb + (k%kin)*sBkk + n*sBn,
 * C(m,n) = C + b*sCb + m*sCm + n (element strides).  a_kcontig: sAkk == 1
 * (else sAm == 1); b_ncontig: sBn == 1 (else sBkk == 1).  kin must be a
 * multiple of 16 (32 for TT_BF16, which reads uint16 bfloat16 A/B and writes
 * float C).  strides[10] = {sAb,sAm,sAkb,sAkk, sBb,sBkb,sBkk,sBn, sCb,sCm, ...}. */
int tt_gemm_dev(void* ctx, int prec, int M, int N, int K, int batch, int kin, const long long* strides, int a_kcontig,
                int b_ncontig, double alpha, double beta, const void* A, const void* B, void* C);

/* Energy E = <x|H_eff|x> (FP64) and its gradients with respect to x, the two
 * environments and the two MPO cores (dense gradient of each sparse entry's
 * 4x4 operator).  Shapes as in tt_heff_apply_dev; gx [rl][4][4][rr],
 * gL [RA][rl][rl], gR [RC][rr][rr] device; gops1/gops2 host [nnz][16]. */
int tt_heff_energy_grad_dev(void* ctx, int rl, int rr, int RA, int RB, int RC, const double* Lenv,
                            const double* Renv, int nnz1, const int32_t* A1, const int32_t* B1, const double* ops1,
                            int nnz2, const int32_t* A2, const int32_t* B2, const double* ops2, const double* x,
                            double* E, double* gx, double* gL, double* gR, double* gops1, double* gops2);

/* Gradient of E = <U|H|U> (current normalised iterate, fixed) with respect to
 * every entry of every MPO core: gops[k] host [nnz_k][16].  Environments are
 * recomputed, not stored, outside the active chain. */
int tt_energy_mpo_grad(void* ctx, double* E, double* const* gops);

/* Per-kernel timing of the effective-Hamiltonian products (HIP events on the
 * library stream).  enable != 0 turns recording on for subsequent products.
 * stats (may be NULL) receives TT_KT_SLOTS rows [ms, launches, algorithmic
 * flops, algorithmic bytes] for the kernels: 0 L.x GEMM; 1, 2, 3 site-1 mix
 * (gather of the rows with few operator entries, GEMM of the rows with many,
 * scatter of those); 4, 5, 6 the same for site 2; 7 R GEMM; 8 its K-split
 * reduction.  With tt_opts.precontract = 1, slot 0 is the GEMM with the left operator
 * (slots 1-3 unused); with precontract = 2, slot 0 is that GEMM into the panels, 7 the
 * panels x right-operator GEMM and 8 its reduction (slots 1-6 unused).  The forming of
 * the operators (once per window) is not in the stats.  One-site products
 * (tt_opts.one_site) use 0 (stage 1: L.x), 1 (light
 * rows of the mix), 2 (GEMM of the heavy rows), 3 (their mix pass), 7 (the
 * products with the stacked right environment) and 8 (their K-split reduction).  Algorithmic work counts only the quantum-number-allowed blocks
 * (block-sparse product) and each operand element moved once.  reset != 0
 * clears the accumulators after copying. */
#define TT_KT_SLOTS 9
int tt_kernel_timing(void* ctx, int enable, double* stats, int reset);

#ifdef __cplusplus
}
#endif

#endif /* TT_H */
