// Device kernels of the additive two-level DMRG hot path (gfx950).
// Internal interface between the kernels and the host orchestration; the
// public C ABI is include/tt.h.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <vector>

namespace tt {

// Failures that the C ABI reports as TT_EHIP: a HIP runtime call, and a
// rocSOLVER/rocBLAS call that returned a bad status.
struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct SolverError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

enum class Prec : int { F64 = 0, F32 = 1, BF16 = 2 };

// Operand addressing of the strided GEMM.  A(m,k), B(k,n) and C(m,n) are
//   A(m,k) = A + batch*sAb + m*sAm + (k / kin)*sAkb + (k % kin)*sAkk
//   B(k,n) = B + batch*sBb + (k / kin)*sBkb + (k % kin)*sBkk + n*sBn
//   C(m,n) = C + batch*sCb + m*sCm + n          (row-major output)
// The contiguous direction of each operand is a template choice:
//   a_kcontig: sAkk == 1 (else sAm == 1);  b_ncontig: sBn == 1 (else sBkk == 1).
// kin must be a multiple of 16 (bond dimensions are padded to 16).
struct GemmArgs {
  int M, N, K, batch;
  int kin;
  long long sAb, sAm, sAkb, sAkk;
  long long sBb, sBkb, sBkk, sBn;
  long long sCb, sCm;
  double alpha, beta;
  // structural-zero skipping (optional; all zero = dense):
  //  kmode 0: full K.
  //  kmode 1: ktab[(batch*mtiles + mtile)*2 + {0,1}] = [lo, hi) range of K.
  //  kmode 2: K = (kb, inner) with nkb outer blocks of kin; ktab[(ntile*nkb + kb)*2 + {0,1}]
  //           = [lo, hi) inner range of block kb for output column tile ntile.
  //  skip: skip[(batch*mtiles + mtile)*ntiles + ntile] != 0 -> the output tile is zero.
  int kmode, nkb, mtiles, ntiles;
  const int* ktab;
  const unsigned char* skip;
};
constexpr int GEMM_TILE = 128;

// C = alpha * A B + beta * C for T in {double, float}.  Accumulation in T.
template <typename T>
void gemm(const GemmArgs& g, const T* A, const T* B, T* C, bool a_kcontig, bool b_ncontig, hipStream_t s);

// Independent row-major GEMMs (a_kcontig, b_ncontig, batch 1) in one launch.
// dev_groups is the device copy of host_groups (used for the launch shape).
template <typename T>
struct GemmGroup {
  GemmArgs g;
  const T* A;
  const T* B;
  T* C;
};
template <typename T>
void gemm_grouped(const GemmGroup<T>* dev_groups, const std::vector<GemmGroup<T>>& host_groups, hipStream_t s);

// The same for problems with few rows (M <= kSkinnyMaxM), row-major, alpha = 1, beta = 0:
// C = A B streamed over B's columns (each thread owns one to four columns and keeps all
// M rows of its columns in registers; A is staged through LDS in K chunks).  Every
// element of B is read once; the cost is B's bytes, not an M-row matrix-core tile.
constexpr int kSkinnyMaxM = 64;
// smallest supported row bucket that holds M rows (16, 32 or 64), 0 if none
int skinny_rows(int M);
template <typename T>
void gemm_grouped_skinny(const GemmGroup<T>* dev_groups, const std::vector<GemmGroup<T>>& host_groups, int mr,
                         hipStream_t s);

// BF16 operands (uint16 storage), FP32 accumulation and FP32 output.
void gemm_bf16(const GemmArgs& g, const uint16_t* A, const uint16_t* B, float* C, bool a_kcontig,
               bool b_ncontig, hipStream_t s);

// Sparse MPO application along one site index:
//   out[c][o][s'][i] = sum_{e in [ptr[c], ptr[c+1])} sum_s op[e][s'][s] * in[src[e]][o][s][i]
// in/out channel slabs have O*4*I elements; channel strides are given so the
// same kernel serves every stage.  op is stored [e][4][4] in the compute type.
// Optional charge tables for structural-zero skipping of the mix: an output
// element (c, o, *, i) can be non-zero only if qi[i] - qo[o] + sgn*qc[c] is the
// charge of a local state; otherwise it is written as zero without gathering.
struct MixQ {
  const int2* qo = nullptr;
  const int2* qi = nullptr;
  const int2* qc = nullptr;
  int sgn = 1;
};
template <typename T>
void mix(int nout, const int* ptr, const int* src, const T* op, const T* in, long long in_cstride,
         T* out, long long out_cstride, int O, int I, hipStream_t s, const MixQ* q = nullptr);

// Elementwise / reduction helpers (double unless noted).
void fill(void* p, size_t bytes, hipStream_t s);                     // zero fill (kernel, graph-safe)
void scale(double* x, double a, size_t n, hipStream_t s);
void axpy(double* y, double a, const double* x, size_t n, hipStream_t s);
void axpby(double* z, double a, const double* x, double b, const double* y, size_t n, hipStream_t s);
void mask_apply(double* x, const uint8_t* mask, size_t n, hipStream_t s);
// out[i] = in[idx[i]] for i < nc, 0 for nc <= i < ncp (compressed vector of a tensor's kept entries)
void gather_idx(double* out, const double* in, const int* idx, size_t nc, size_t ncp, hipStream_t s);
// out[idx[i]] = in[i] for i < nc (other entries of out untouched)
void scatter_idx(double* out, const double* in, const int* idx, size_t nc, hipStream_t s);
// out[i] = sum_n V[i*ldv + n] * w[n] for i < m  (deterministic two-pass reduction).
// partial holds at least cap_blk * m doubles; the first pass uses dot_blocks(n) workgroups,
// at most cap_blk (the summation order depends on n and cap_blk only).
constexpr int kDotBlocks = 1024;
int dot_blocks(size_t n);
void multi_dot(const double* V, size_t ldv, int m, const double* w, size_t n, double* out_dev, double* partial,
               int cap_blk, hipStream_t s);
// Batched one-sided Jacobi SVD of tall matrices (M >= N, column-major with leading
// dimension lda), one workgroup per matrix.  A is overwritten; V is an N x N scratch
// (unused when the matrix is held in LDS: in_lds requires (M + N) N <= kJacobiLds).  On
// exit S[0..N) holds the singular values in decreasing order, U (leading dimension ldu) the
// left and Vt (leading dimension ldvt) the right singular vectors; info = 0, 1 where the
// sweeps did not converge, -1 for a shape the kernel does not take.
struct SvdJob { double* A; double* V; double* U; double* S; double* Vt; int* info; int M, N, lda, ldu, ldvt, pad; };
constexpr int kJacobiMaxN = 1024;
constexpr int kJacobiLds = 17920;  // doubles of A and V held in LDS (140 KiB)
void jacobi_svd(const SvdJob* jobs, int njobs, int max_sweeps, bool in_lds, hipStream_t s);
// Blocked Jacobi SVD of the same matrices (same outputs and info), each spread over many
// workgroups: columns in blocks of 8, one launch for the pairs inside the blocks and one per
// round of a tournament over the blocks, every column pair once per sweep; the host reads
// the per-matrix rotation counts after each sweep (one stream synchronisation per sweep).
// V must be an N x N scratch.  jacobi_blocked_fits: the launches can hold two blocks'
// columns of A and V in LDS (M + N <= 1152).  rows: rows per lane the pair kernels hold in
// registers (4 or 9; 0 = loops over LDS; -1 = the fewest that cover the largest M).  fro2,
// rot and act_dev are device scratch of njobs entries each.
bool jacobi_blocked_fits(int M, int N);
void jacobi_svd_blocked(const SvdJob* jobs, const SvdJob* jobs_host, int njobs, int rows, int max_sweeps,
                        double* fro2, int* rot, int* act_dev, hipStream_t s);
// out[n] = sum_i c[i] V[i*ldv+n]  (c on device)
void lincomb(const double* V, size_t ldv, int m, const double* c_dev, double* out, size_t n, hipStream_t s);
void convert_f64_f32(const double* a, float* b, size_t n, hipStream_t s);
void convert_f32_f64(const float* a, double* b, size_t n, hipStream_t s);
void convert_f64_bf16(const double* a, uint16_t* b, size_t n, hipStream_t s);
// FP32 copy holding the bfloat16 rounding (round to nearest even) of each value
void convert_f64_bf16f32(const double* a, float* b, size_t n, hipStream_t s);
void convert_f64_f32_op(const double* a, float* b, size_t n, hipStream_t s);
// gather / scatter of a 2-D block: dst[i*ldd + j] = src[rows[i]*lds + cols[j]] (column-major dst if colmajor)
void gather2d(const double* src, long long lds, const int* rows, int nr, const int* cols, int nc, double* dst,
              bool colmajor, hipStream_t s);
// dst[rows[i]*ldd + cols[j]] = alpha * src[i*sr + j*sc] * (rs ? rs[i] : 1) * (cs ? cs[j] : 1)
// tri: 0 full, 1 keep i <= j (upper), 2 keep j <= i (lower); other entries written as 0
void scatter2d(const double* src, long long sr, long long sc, const int* rows, int nr, const int* cols, int nc,
               double* dst, long long ldd, double alpha, const double* rs, const double* cs, int tri, hipStream_t s);
// Core with permuted bonds: out[a][s][b] = in[pl[a]][s][pr[b]] for a < rl, b < rr
// (padded strides irp/orp of the right bonds); other entries of out are left alone.
void permute_core(const double* in, int irp, const int* pl, const int* pr, int rl, int rr, double* out, int orp,
                  hipStream_t s);
// copy a strided 3-D block: dst[i*d0 + j*d1 + k] = alpha * src[i*s0 + j*s1 + k]
// (accumulate: dst[...] += alpha * src[...])
void copy3d(const double* src, long long s0, long long s1, double* dst, long long d0, long long d1, int n0, int n1,
            int n2, double alpha, hipStream_t s, bool accumulate = false);

// Batched block gather / scatter of the sector-wise factorisations.
// gather: dst[b.dst + j*b.ld + i] = M[rows[b.roff+i]*ldm + cols[b.coff+j]]  (column-major blocks);
// with b.trans the block is stored transposed: dst[b.dst + i*b.ld + j] for i < m, j < n
struct GatherBlk { long long dst; int ld, roff, coff, m, n, trans; };
void gather_blocks(const double* M, long long ldm, const int* rows, const int* cols, const GatherBlk* blks, int nblk,
                   double* dst, hipStream_t s);
// scatter of kept factors: for block b with t kept vectors starting at bond index off,
//   left [rows[roff+i]*ldl + off + j] = U[i*us_i + j*us_j] * (mode == 1 ? S[j] : 1)      i < m, j < t
//   right[(off + j)*ldr + cols[coff+c]] = Vt[j*vs_j + c*vs_c] * (mode == 0 ? S[j] : 1)   j < t, c < n
struct ScatterBlk {
  const double* U;
  const double* Vt;
  const double* S;
  long long us_i, us_j, vs_j, vs_c;
  int roff, coff, m, n, t, off;
};
// Householder LQ of charge-sector blocks, one workgroup per block.  Block b is
//   B[r][c] = W[rows[roff+r]*sWr + cols[coff+c]*sWc]   (m x n, k = min(m, n))
// factored as B = L Q with reflectors applied from the right (LAPACK convention:
// Q = first k rows of H(k-1)...H(0), H(i) = I - tau_i v_i v_i^T, v_i[i] = 1), then
//   Lout[rows[roff+r]*sLr + nmap[noff+c]*sLc] = L[r][c]   for c <= min(r, k-1)
//   Qout[nmap[noff+r]*sQr + cols[coff+c]*sQc] = Q[r][c]   for r < k
// (nmap: bond index of each factor row; other destination entries untouched).
// ws + b.ws holds the block's m x n working copy, then its k x n Q, then its k
// reflector scales.  n <= HH_MAXN.
struct HhBlk { long long ws; int m, n, roff, coff, noff, pad; };
constexpr int HH_MAXN = 6144;
void householder_lq(const double* W, long long sWr, long long sWc, const int* rows, const int* cols, const int* nmap,
                    const HhBlk* blks, int nblk, double* ws, double* Lout, long long sLr, long long sLc, double* Qout,
                    long long sQr, long long sQc, hipStream_t s);
void scatter_factors(const ScatterBlk* blks, int nblk, const int* rows, const int* cols, double* left, long long ldl,
                     double* right, long long ldr, int mode, hipStream_t s);

// gop[e][s'][s] += sum_{o,i} G[cg(e)][o][s'][i] * T[ct(e)][o][s][i] for every entry e
// (entries given as flat lists; one workgroup per entry, deterministic reduction)
template <typename T>
void entry_grad(int nnz, const int* gch, const int* tch, const T* G, long long g_cs, const T* Tin, long long t_cs,
                int O, int I, double* gop, hipStream_t s);
// batched transpose of [n][r][c] -> [n][c][r]
void transpose_batched(const double* in, double* out, int n, int r, int c, hipStream_t s);

// diagonal of the effective Hamiltonian: env diagonals, channel mixes of the
// diagonal local-operator elements, preconditioner application
void diag_extract(const double* E, int R, int r, double* out, hipStream_t s);
void diag_mix(int nout, const int* ptr, const int* src, const double* op, const double* in, int n, double* out,
              bool state_inner, hipStream_t s);
// t = r / (theta - d), |theta - d| clamped to >= 1e-3, where m (may be null: every entry) is set
void precond(double* t, const double* r, const double* d, double theta, const uint8_t* m, size_t n, hipStream_t s);

}  // namespace tt
