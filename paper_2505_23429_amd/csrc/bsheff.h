// Quantum-number block-sparse form of the two-site effective-Hamiltonian
// product of one window (sites k, k+1).
//
// Bond labels are grouped by charge into sectors (alpha on the left bond,
// beta on the right bond).  The channel index and one site index of every
// intermediate combine into a row (K, s) whose charge Gamma = q(s) - d_K is
// conserved by each MPO site tensor; the remaining indices form a spectator
// block (alpha', s_other, beta) of shape n_alpha' x n_beta, and a spectator
// belongs to the group Gamma = Q_beta - Q_alpha' - q(s_other).  Per group an
// intermediate is one dense row-major matrix [rows x spectator elements], so
//   stage 1  T1 = L_A x           grouped GEMM per left sector alpha
//   mix 1    T2 = W1 T1           sparse x dense product per group (site k)
//   mix 2    T3 = W2 T2           sparse x dense product per group (site k+1)
//   stage 4  y  = sum_C T3 R_C^T  grouped split-K GEMM per right sector beta'
// store and touch only the structurally non-zero entries.  The environments
// stay dense; x and y are the dense padded vectors [rlp][4][4][rrp].
//
// Stage 1 and mix 1 can instead run as one GEMM on a precontracted left operator
//   LW[(B, s1', alpha', i')][(s1, a)] = sum_A W1[A, s1', s1, B] L_A[alpha' + i'][alpha + a]
// (alpha' = alpha + d_A), which depends on the window only and is formed once per
// window.  Its rows are grouped by the charge gamma = alpha + q(s1) = alpha' + q(s1')
// - d_B of the ket's left half and by the set of site states s1 with a non-zero
// operator entry in row s1' of channel B (the mask); per group
//   T2[(B, s2)][spec(alpha', s1', beta) + i' n_beta + j] = sum_(s1, a) LW x[a][s1][s2][j],
// beta = gamma + q(s2): T1 is never formed, and the heavy rows of W1 (the
// accumulating channels) are summed once per window instead of once per product.
//
// With the right operator precontracted as well,
//   WR[(B, s2, b)][j'] = sum_C W2[B, s2', s2, C] R_C[beta' + j'][beta + b]
// (also formed once per window), the rest of the product is one split-K GEMM per
// panel (zeta, s2'): zeta = alpha' + q(s1') is the charge of the bra's left half, the
// panel's rows are (s1', alpha' = zeta - q(s1'), i') and its K runs over the chunks
// (B, s2, b) whose operator entries reach s2' (beta = zeta - d_B + q(s2),
// beta' = zeta + q(s2')); the left-operator GEMM writes each of its outputs once, into
// the chunk store of its zeta that the panels read, and y[alpha', s1', s2', beta'] =
// panel x WR.  T2 as rows (B, s2), the second mix and T3 are then never formed either.
#pragma once
#include "engine.h"

namespace tt {

struct BsAlpha { int M, N, K, row0, col0, oal; };
// ld: row stride (ncols rounded up to 4); cls[s]: charge class of the output
// channels of rows with site state s in the second mix (-1: none)
struct BsGroup { long long in_base; int ncols, spec0, nspec, ld; int cls[4]; };
// One output row of a mix.  First mix: b[s] is the T2 row base for spectator
// site state s; sy is the output site state s1'.  Second mix: sy is s2' and
// rank the position of the output channel within its charge class (its K
// offset in a stage-4 panel is the sector start + rank * n_beta).  Light rows
// read operator entries [e0, e1); heavy rows read the staging row at h.
struct MixRow { long long b[4]; long long h; int e0, e1, sy, rank, pad0, pad1; };
// One mix workgroup: group g, spectator columns [c0, c0 + 256), output rows [r0, r1).  When
// ns > 0 the distinct input rows its rows read are stage[s0 .. s0 + ns) and are loaded once
// into LDS; operator entry e then reads staged row oloc[e].
struct MixTile { int g, c0, r0, r1, s0, ns, pad0, pad1; };
struct BsS4Tile { long long abase, bbase; int M, N, K, m0, n0, k0, k1, slot; };
struct BsRedTile { int M, N, m0, n0, slot0, nsplit, row0, pad; };
struct BsPair { int C, beta, koff, bprime; };
// One GEMM of the precontracted left operator: rows [0, M) (row blocks [rb0, rb0 + nrb)),
// LW rows at a0 with stride K4 (K rounded up to 8; the padding is zero), K entries of the
// x-row table from k0 (pieces: site state ps, first k pk, length pn, ket sector pa), N
// columns of the column table from n0 ({x offset, s2 << 20 | j}), right sector be[s2].
struct BsLwGroup {
  long long a0;
  int M, K, K4, N, k0, n0, rb0, nrb, np, pad;
  int be[4], ps[4], pk[4], pn[4], pa[4];
};
// rows [r0, r0 + n) of group g: output channel and bra state bs = B * 4 + s1', bra sector
// ap; with the right operator, zi indexes the block's zeta and kci the chunk table
// (entries [kci * 4 + s2]: the first column of the chunk (B, s2) in the zeta's store, -1 none)
struct BsLwBlock { int g, r0, n, bs, ap, zi, kci, pad; };
// the chunks of one zeta: M rows (s1', alpha', i') from row0[s1'] (-1: no alpha'); every
// chunk (B, s2) that a panel of this zeta uses is stored once, at zbase + kc M as the
// row-major block [M][nb8] (nb8 = n_beta rounded up to 8, the padding zero), so that an
// output block of the left-operator GEMM is contiguous and written once
struct BsZeta { long long zbase; int M, row0[4], pad; };
// one panel (zeta, s2'): rows M, K columns (its chunks, each padded to 8), N = n_beta'; its
// A operand is read from the zeta's chunks (from pbase, the zeta's store) through the
// column table, WR at wbase is [K][N]
struct BsPanel { long long pbase, wbase; int M, K, N, zi, s2p, bep, pad0, pad1; };
// per 8 panel columns: the offset of their chunk columns from zbase for row 0, and the
// chunk's row stride
struct BsK8 { int off, nb8; };
// one workgroup of the panel GEMM (the stage-4 tile with the panel's column table at t8)
struct BsPTile { long long abase, bbase, t8; int M, N, K, m0, n0, k0, k1, slot; };
// one block of WR: panel P, chunk (B, s2) = bs2 / 4, bs2 % 4 at column kc, right sector be
struct BsWrItem { int P, bs2, kc, be; };
// one workgroup: rows [m0, m0 + 128) of group g, overlapped by row blocks [rb0, rb0 + nrb)
struct BsLwTile { int g, m0, rb0, nrb; };

// One sparse x dense mix.  Output rows with few operator entries ("light",
// nearly all of them) are gathered entry by entry; the few rows with many
// entries ("heavy": the accumulating channels, whose rows are almost dense
// within their group) form a dense [H x rows_in] matrix per group applied by
// the MFMA GEMM into a staging buffer, then scattered like the light rows.
struct BsHeavy { int g, H, Nin, Nin4, cols, ld; long long in_base, w_off, tmp_off; };
struct BsMix {
  int ntiles = 0, nhtiles = 0, nstage = 0, noloc = 0, nstaged = 0;  // nstaged: light tiles that stage
  double flops = 0.0, nin = 0.0, nout = 0.0;  // algorithmic flops; elements read and written once
  // per kernel: gather of the light rows, GEMM and scatter of the heavy rows (flops, elements)
  double fl_light = 0.0, el_light = 0.0, fl_heavy = 0.0, el_heavy = 0.0, el_scatter = 0.0;
  long long ntmp = 0;                         // staging elements of the heavy rows
  std::vector<BsHeavy> heavy;
  DevMem tiles, groups, rows, ocol, oval64, oval32, spec, stage, oloc;
  DevMem htiles, hrows, hw64, hw32;
};

struct BsPlan {
  bool ok = false;
  long long serial = 0;
  int rlp = 0, rrp = 0, nal = 0, nbe = 0, RAx = 0, RB = 0, RC = 0, RCx = 0, ndcls = 0;
  long long n1 = 0, n2 = 0, n3 = 0, nrs = 0;  // elements of T1, T2, T3 and the stacked R
  double flops1 = 0.0, flops4 = 0.0;          // block-sparse flops of stages 1 and 4
  double bytes1 = 0.0, bytes4 = 0.0;          // element counts moved once by stages 1 and 4
  double el_red = 0.0;                        // elements moved by the stage-4 reduction
  // stage 1
  int ntiles1 = 0;
  DevMem tiles1, alpha, rsrc, rinfo, cinfo, rowpart1, specoff, nbeta, boff;
  // mixes
  BsMix m1, m2;
  DevMem bshift, pbase, kbeta, kstart;  // second-mix destinations: class x sector -> panel, panel bases, K starts
  // stage 4
  int ntiles4 = 0, nred = 0, nslots = 0, npairs = 0;
  DevMem tiles4, red, rowdst, pairs, rbase;
  DevMem rstack64, rstack32;
  bool have64 = false, have32 = false;
  // precontracted left operator (lw): replaces stage 1 and mix 1
  bool lw = false;
  int nlw_groups = 0, nlw_tiles = 0, nlw_blocks = 0;
  long long nlw = 0;                       // elements of LW
  double flops_lw = 0.0, bytes_lw = 0.0;   // per product: flops; elements of LW, x read and T2 written
  double build_lw = 0.0;                   // multiply-adds of forming LW (once per window)
  DevMem lw_groups, lw_tiles, lw_blocks, lw_krow, lw_col, lw_tptr, lw_tA, lw_tv, rowbase2, aoff;
  DevMem lw64, lw32;
  bool have_lw64 = false;
  int lw32_state = 0;                      // LW in FP32: 0 not formed, 1 rounded to FP32, 2 to bfloat16
  // precontracted right operator (wr, with lw): panels replace T2, mix 2, T3 and stage 4's panels
  bool wr = false;
  int nwr_items = 0, npanels = 0;
  long long nwr = 0;                       // elements of WR (n2: elements of the chunk stores)
  double build_wr = 0.0;                   // multiply-adds of forming WR
  DevMem lw_zeta, lw_kc, wr_items, wr_panels, wr_tptr, wr_tC, wr_tv, wr64, wr32, wr_k8, wr_ptiles;
  DevMem lw16, wr16;                       // bfloat16 copies of LW and WR (bf16 products)
  bool have_lw16 = false, have_wr16 = false;
  int nptiles = 0;
  long long nk8 = 0;
  int wr32_state = 0;
  DevMem err;  // set by a kernel when an index would leave its buffer (the access is skipped)
};

// Builds the plan of the window at sites (b, b+1).  Returns false (no plan)
// when the labels of a bond are not grouped by charge.
bool bs_build(Engine& E, BsPlan& p, int b, const Labels& ql, const Labels& qr, int rlp, int rrp, int RAx, int nP);

// y = H_eff x.  L: [RAx][rlp][rlp] (virtual channels included), R: [RC][rrp][rrp],
// Rt: [RCx - RC][rrp][rrp] (second-site block channels), x, y: [rlp][4][4][rrp].
// bf16_t3 rounds the mix-2 output to bfloat16 before the last contraction.
// check = false: launches only (graph capture); bs_check then reads the plan's index check.
template <typename T>
void bs_apply(Engine& E, BsPlan& p, const T* L, const T* R, const T* Rt, const T* x, T* y, bool bf16_t3,
              bool check = true);
void bs_check(Engine& E, BsPlan& p);
// Forms the precontracted operators of a plan with p.lw (FP64): LW from the environment
// L [RAx][rlp][rlp] (nL elements) and, with p.wr, WR from R [RC][rrp][rrp] and the block
// channels Rt [RCx - RC][rrp][rrp]; the FP32 copies follow on first use.
void bs_lw_build(Engine& E, BsPlan& p, const double* L, long long nL, const double* R, const double* Rt);

// ---------------------------------------------------------------------------
// Block-sparse environment update through one site (FP64).
//   left  (sigma = +1): out[B][b'][b] = sum E[A][a'][a] Ubra[a'][s'][b'] W[A,s',s,B] Uket[a][s][b]
//   right (sigma = -1): out[A][a'][a] = sum Ubra[a'][s'][b'] W[A,s',s,B] Uket[a][s][b] E[B][b'][b]
// Rows (channel, s) of the intermediates are grouped by Gamma = sigma q(s) - d,
// conserved by the site operator; spectators are (bra sector at the input
// bond, ket sector at the output bond).  The charge-grouped operator tables
// depend only on the site and are built once per MPO.
// ---------------------------------------------------------------------------
struct BsSiteUse {
  int sigma = 1, nin = 0, nout = 0, ncin = 0, ncout = 0, ngrp = 0;
  std::vector<Q2> cq_in, cq_out;           // class charges
  std::vector<int> cls_in, cls_out;        // class of every channel
  std::vector<int> cstart_in, cstart_out;  // class -> first entry of clist (size nc + 1)
  std::vector<int> gidx_in;                // [nin*4] row group of (channel, s), -1 if none
  std::vector<Q2> gq;                      // group charges
  std::map<Q2, int> gid;
  std::vector<int> orow0;                  // group -> first output row (size ngrp + 1)
  std::vector<int> nrows_in;               // input rows per group
  std::vector<double> nent_light;          // operator entries of the light output rows per group
  double nnz = 0.0;                        // operator non-zeros (for flop counts)
  DevMem clist_in, clist_out, pos_out, d_cls_out, d_gidx_in, rin, optr, ocol, oval, orow;
  // heavy output rows (many entries) as a dense [H x rows_in] matrix per group
  std::vector<int> hrow0;                  // group -> first heavy row (size ngrp + 1)
  std::vector<int> nin4;                   // rows_in rounded up to 4 (row stride of the dense matrix)
  std::vector<long long> hw_off;           // group -> offset of its dense matrix
  DevMem hrow, hw;
};

// Builds the site tables: op grouped by output channel (nout outputs, inputs
// < nin) with channel charges din/dout; sigma as above.
void bs_site_use(Engine& E, BsSiteUse& u, const SiteOp& op, const std::vector<Q2>& din,
                 const std::vector<Q2>& dout, int sigma);

// One update.  Ein: [nin][Pp][Qp] at the input bond (bra rows P, ket columns Q);
// bra/ket: the two cores; out: [nout][Tp][Rp] (bra T, ket R) at the output bond,
// overwritten.  Returns false when a bond's labels are not grouped by charge
// (the caller then uses the dense update).
bool bs_env(Engine& E, const BsSiteUse& u, const double* Ein, const Core& bra, const Core& ket, double* out);

// ---------------------------------------------------------------------------
// One-site effective-Hamiltonian product (eq. mat_vec, one-site form, FP64):
//   y[a'][s'][b'] = sum L[A][a'][a] W[A,s',s,B] x[a][s][b] R[B][b'][b]
// through stage 1 and the mix of the left update (ket = x), then split-K products
// of each right sector's panel with the right environment stacked for that sector.
// use: the left-update tables of the site (virtual input channels at a block site,
// whose L then carries them); ql/qr: bond labels of x (grouped by charge);
// R: [RB][rrp][rrp], read once by the build.  x, y: [rlp][4][rrp]; y is overwritten.
// ---------------------------------------------------------------------------
// Split-K products of row panels with stacked matrices whose rows are scattered into
// y (the kernels of the two-site product's last stage): segment g multiplies the
// panel [M][K] at abase by the stacked [K][N] at bbase, and its row m lands at
// y[rowdst[row0 + m] + n].  part holds 64 x 64 doubles per slot.
struct BsSplitSeg { long long abase, bbase; int M, N, K, row0; };
void bs_splitk_tables(const std::vector<BsSplitSeg>& segs, std::vector<BsS4Tile>& tiles, std::vector<BsRedTile>& red,
                      int& nslots, double& el_red);
void bs_splitk_run(Engine& E, int ntiles, const BsS4Tile* tiles, int nred, const BsRedTile* red,
                   const long long* rowdst, const double* A, long long nA, const double* B, long long nB, double* part,
                   double* y, long long ny, int* err, int slot_gemm, int slot_red);
constexpr int kBsSplitTile = 64;

struct BsHeff1Impl;
struct BsHeff1 {
  std::shared_ptr<BsHeff1Impl> p;
  double flops = 0.0;  // block-sparse flops of the two contractions of one product
};
bool bs_heff1_build(Engine& E, BsHeff1& h, std::shared_ptr<BsSiteUse> use, const Labels& ql, const Labels& qr, int RAx,
                    const double* R, int RB);
void bs_heff1_apply(Engine& E, BsHeff1& h, const double* Lx, const double* x, double* y);

}  // namespace tt
