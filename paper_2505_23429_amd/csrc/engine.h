// Host-side engine of the additive two-level DMRG hot path: device tensors,
// sparse MPO cores, environments, sector-wise linear algebra (rocSOLVER),
// Davidson and the four steps of one global iteration.
#pragma once
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <array>
#include <climits>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/tt.h"
#include "kernels.h"

namespace tt {

constexpr int PAD = 32;  // every bond dimension is stored padded to a multiple of 32
inline int padr(int r) { return ((r + PAD - 1) / PAD) * PAD; }

using Q2 = std::array<int, 2>;
using Labels = std::vector<Q2>;

// a device allocation that neither the large-block arena nor the block pool could serve
struct DeviceOOM : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// Device allocator supplied by the caller (tt_opts.dev_alloc/dev_free/alloc_user).
struct ExtAlloc {
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*free)(void*, void*, void*) = nullptr;
  void* user = nullptr;
};
// Allocator (nullptr: the library's pools) and stream that new blocks of the call
// running on this thread come from / will be used on.
void set_thread_allocator(const ExtAlloc* a, hipStream_t s);

struct DevMem {
  void* p = nullptr;
  size_t n = 0;      // bytes in use
  size_t cap = 0;    // bytes allocated (pooled block)
  bool own = true;   // false: a caller's buffer, never freed here
  const ExtAlloc* ext = nullptr;  // the caller's allocator this block came from, if any
  hipStream_t ext_stream = nullptr;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept : p(o.p), n(o.n), cap(o.cap), own(o.own), ext(o.ext), ext_stream(o.ext_stream) {
    o.p = nullptr; o.n = 0; o.cap = 0; o.own = true; o.ext = nullptr; o.ext_stream = nullptr;
  }
  DevMem& operator=(DevMem&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; cap = o.cap; own = o.own; ext = o.ext; ext_stream = o.ext_stream;
      o.p = nullptr; o.n = 0; o.cap = 0; o.own = true; o.ext = nullptr; o.ext_stream = nullptr;
    }
    return *this;
  }
  void borrow(void* q, size_t bytes) { release(); p = q; n = bytes; cap = bytes; own = false; }
  ~DevMem() { release(); }
  void release();
  void ensure(size_t bytes);       // grow-only, contents not preserved
  void resize_zero(size_t bytes, hipStream_t s);  // exact size, zero filled
  template <class T> T* as() const { return (T*)p; }
};

// A TT core on the device: f64 [rlp][4][rrp], zero padded.
struct Core {
  int rl = 0, rr = 0;
  Labels ql, qr;
  DevMem d;
  int rlp() const { return padr(rl); }
  int rrp() const { return padr(rr); }
  size_t elems() const { return (size_t)rlp() * 4 * rrp(); }
};

// One CSR form of a sparse MPO core (grouped by output channel).
struct SiteOp {
  int nout = 0, nnz = 0;
  DevMem ptr, src, op64, op32;
  std::vector<int> hptr, hsrc;   // host copy of the CSR (grouped by output channel)
  std::vector<double> hop;       // [nnz][4][4]
};

struct BsSiteUse;  // block-sparse environment-update tables of one site (bsheff.h)

struct SiteMPO {
  int Rl = 0, Rr = 0;
  std::vector<int> A, B;          // all entries (host)
  std::vector<double> ops;        // [nnz][16]
  SiteOp byB, byA;                // all entries
  bool has_block = false;
  int p0 = 0, p1 = 0, q0 = 0, q1 = 0;
  DevMem V;                       // [q1-q0][p1-p0] f64 coefficient block
  // the coefficient block per channel charge class (it only couples channels of equal
  // charge): block-relative input channels P, output channels Q, V restricted to them
  struct VClass {
    Q2 d;
    std::vector<int> P, Q;
    DevMem Pd, Qd, V;  // ints, ints, [|Q|][|P|]
  };
  std::vector<VClass> vcls;
  SiteOp byB_left;                // block -> virtual pass entries (inputs Rl + q - q0)
  SiteOp byB_noblk;               // block entries removed
  SiteOp byA_right;               // block -> virtual pass entries (inputs Rr + p - p0)
  SiteOp byB_rightv;              // block entries replaced by outputs Rr + (p - p0) (second site of a window)
  std::shared_ptr<BsSiteUse> bs_left, bs_right;  // built on first block-sparse environment update
};

// Structural-zero tables of one two-site window (device arrays).
struct WinTabs {
  DevMem k1tab, k1skip;   // stage 1: [RAx][mtiles][2] K ranges, [RAx][mtiles][ntiles] zero tiles
  int m1tiles = 0, n1tiles = 0;
  DevMem k4tab;           // stage 4: [ntiles][RC][2] inner K ranges
  DevMem k4tabP;          // extra stage-4 GEMM of the second-site block: [ntiles][nP][2]
  int n4tiles = 0;
  DevMem qo1, qi1, qo2, qi2;            // int2 charge arrays of the two mixes
  const int2* qcB = nullptr;            // channel charges of the middle bond (not owned)
  const int2* qcC = nullptr;            // channel charges of the right bond (not owned)
};

struct Env {
  int R = 0, rb = 0, rk = 0;  // true sizes; storage [R][rbp][rkp]
  DevMem d;
  size_t elems() const { return (size_t)R * padr(rb) * padr(rk); }
};

struct Davidson {
  int iters = 0, matvecs = 0;
  int matvecs64 = 0;  // of which FP64 products
  bool converged = false;
  double theta = 0.0, resid = 0.0;
};

// The operator and its device tables: shared (read-only during the local solves)
// between a context and the worker engines that run subdomain solves concurrently.
struct Problem {
  int L = 0;
  std::vector<SiteMPO> mpo;
  std::vector<int> Rb;                 // bond dims
  std::vector<Labels> chan_q;          // per bond
  std::vector<DevMem> chan_q_dev;      // per bond, int2
  std::mutex mu;                       // guards the lazily built per-site tables
};

class Engine {
 public:
  explicit Engine(const tt_opts& o);
  // worker engine: own stream, rocBLAS handle, workspaces and counters; the
  // problem is the parent's
  Engine(const Engine& parent, int worker);
  ~Engine();
  tt_opts opts;
  hipStream_t stream = nullptr;
  bool own_stream = true;     // false: the caller's stream (tt_opts.stream)
  void* noalloc = nullptr;    // device address of this device's no-allocation scratch array
  ExtAlloc ext;               // the caller's allocator (alloc == nullptr: the library's pools)
  rocblas_handle blas = nullptr;
  std::string err;

  // problem
  std::shared_ptr<Problem> prob;
  int& L;
  std::vector<SiteMPO>& mpo;
  std::vector<int>& Rb;
  std::vector<Labels>& chan_q;
  std::vector<DevMem>& chan_q_dev;
  std::vector<Core> U;                 // current left-orthogonal iterate (unit norm)
  // linear-system functional: the iterate is X = xscale * tau(U); F its right-hand side;
  // FL[k] = <U_0..U_{k-1} | F_0..F_{k-1}> at subdomain starts, FR[k] = <V_k..V_{L-1} | F_k..>
  // (one-channel environments [1][r_bra][r_F]); uf = <tau(U)|F>; coarse_b the coarse right-hand side
  double xscale = 1.0, xscale_saved = 1.0;
  std::vector<Core> Fc;
  bool have_rhs = false;
  std::vector<Env> FL, FR;
  double uf = 0.0;
  std::vector<double> coarse_b;
  std::vector<Core> Usaved;            // device copy kept by tt_mps_checkpoint
  bool have_mpo = false, have_mps = false;

  // Step 1 products (valid after local_solve)
  std::vector<Core> Vc, Wc;            // right-orthogonal cores and centres
  std::vector<Env> Lenv, Renv;         // environment caches
  // Step 2 products
  struct Sub {
    int s = 0, t = 0;                  // modified sites [s, t]
    std::vector<Core> mod;             // cores s..t
    double E = 0.0;
    int matvecs = 0, matvecs64 = 0;
    bool converged = true;
    // Extension One: the updates of the same subdomain from its next-lowest local
    // eigenvectors (cores s..t, sharing all but the last two with this one)
    std::vector<Sub> alt;
  };
  std::vector<Sub> subs;                // coarse states 1.. (per subdomain: lowest update, then alternatives)
  std::vector<int> sub_base;            // per subdomain: index in subs of its lowest update
  bool have_local = false;
  // worker engines of the concurrent subdomain solves (created on first use)
  std::vector<std::unique_ptr<Engine>> workers;

  // timing / accounting
  double flops_heff = 0.0, sec_heff = 0.0;
  // wall-clock phases of a sweep (seconds, stream synchronised at each boundary):
  // 0 LQ sweep, 1 step-1 environments, 2 window set-up, 3 Davidson, 4 two-site
  // splits, 5 environment updates of the subdomain sweeps, 6 coarse matrices,
  // 7 coarse eigenproblem and compression, 8 all subdomain solves (wall clock).
  // With concurrent solves, 2-5 are summed over the workers.
  static constexpr int NPH = 9;
  double ph[NPH] = {};
  double now();
  // verbose-mode counters: environment updates (block-sparse, dense) and overlap updates
  double t_env_bs = 0.0, t_env_dense = 0.0, t_ov = 0.0;
  int n_env_bs = 0, n_env_dense = 0, n_ov = 0;
  // verbose mode: batched SVD calls per padded bin shape {M, N} -> {calls, matrices, unused},
  // and the wall time of the batched SVD phases
  std::map<std::pair<int, int>, std::array<double, 3>> svd_bins;
  double svd_seconds = 0.0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int warn = 0;
  bool verbose = false;
  int verbose_level = 0;
  // per-kernel statistics of the effective-Hamiltonian products (tt_kernel_timing):
  // kstat[slot] = {ms, launches, algorithmic flops, algorithmic bytes}; slots
  // 0 L.x GEMM, 1/2/3 site-1 mix (gather, heavy-row GEMM, heavy-row scatter),
  // 4/5/6 site-2 mix (same), 7 R GEMM, 8 R GEMM K-split reduction
  static constexpr int KT_SLOTS = TT_KT_SLOTS;
  bool kt_on = false;
  hipEvent_t kt_ev[KT_SLOTS + 1] = {};
  int kt_slot[KT_SLOTS + 1] = {};
  int kt_n = 0;
  double kstat[KT_SLOTS][4] = {};
  int cur_rl = 0, cur_rr = 0, cur_RA = 0, cur_RC = 0;
  void kt_begin();           // start event of one product
  void kt_mark(int slot);    // closes the interval since the previous event, attributed to slot
  void kt_end(const double* fl, const double* by);  // per-slot algorithmic work of the product

  // setup
  void set_mpo(int L, const int* R, const int* nnz, const int32_t* const* A, const int32_t* const* B,
               const double* const* ops, const int32_t* const* cq, const int* block);
  void set_mps(int L, const int* r, const double* const* Uh, const int32_t* const* q);
  void get_mps(int* r, double* const* Uh, int32_t* const* q);
  double energy();
  double functional_value();  // J(X): Rayleigh quotient, or 1/2 <X,AX> - <F,X>
  void set_rhs(int L, const int* r, const double* const* Fh, const int32_t* const* q);
  double overlap_with_rhs();  // <tau(U)|F>
  // one-channel overlap environments (bra, ket may differ in bond dimensions and labels)
  void ov_left(const Env& in, const Core& bra, const Core& ket, Env& out);
  void ov_right(const Env& in, const Core& bra, const Core& ket, Env& out);
  void checkpoint(int op);  // 0: keep a device copy of the iterate, 1: make it current again

  // algorithm
  void local_solve(int nsub, const int* lengths, double* E, int* mv);
  // Step 2 for one subdomain (sites s..e): this engine's stream and workspaces,
  // the Step-1 cores and environments of src
  void solve_subdomain(const Engine& src, int j, int s, int e, Sub& S);
  void solve_subdomain1(const Engine& src, int j, int s, int e, Sub& S);  // one-site micro-steps
  std::shared_ptr<BsSiteUse> left_site_use(int site);
  void absorb_counters(Engine& w);  // add a worker's counters to this engine's, clear the worker's
  // fn(engine, task) for every task: on this engine in order when one worker is asked
  // for, else on worker engines (host thread + stream each), the costliest tasks first.
  // fn reads shared state only and writes task-private outputs.
  void run_tasks(int ntask, const std::vector<double>& cost, const std::function<void(Engine&, int)>& fn);
  int coarse_correct(double* S, double* A, double* c, double* lam, double* Eout, int* rank, double* disc);
  // Step 4's block TT of sum_j c_j U^j (labels grouped by charge within each block)
  void combination_tt(const std::vector<double>& c, std::vector<Core>& T);
  // the same TT with every bond's labels grouped by charge (a permutation of each bond)
  void grouped_combination(const std::vector<double>& v, std::vector<Core>& W);
  // z = A v with A_ij = <U^i|H|U^j>, through environment chains with the combination TT
  // (the coarse matrix is not formed); returns the number of environment updates
  int coarse_apply(const std::vector<double>& v, std::vector<double>& z);
  int coarse_matvecs = 0;  // Krylov products of the last coarse step
  void dmrg2(int nsweeps, double* energies);

  // kernels on raw device pointers
  template <class T>
  void heff(int rl, int rr, int RA, const T* Lenv, const SiteOp& w1, int RB, const SiteOp& w2, int RC, const T* Renv,
            const T* x, T* y, const T* Rtil, int P0, int nP, const WinTabs* tabs = nullptr);
  void heff_bf16(int rl, int rr, int RA, const uint16_t* Lenv, const SiteOp& w1, int RB, const SiteOp& w2, int RC,
                 const uint16_t* Renv, const uint16_t* x, float* y, const uint16_t* Rtil, int P0, int nP,
                 const WinTabs* tabs = nullptr);
  void env_left_raw(int rb, int rk, int rb2, int rk2, int RA, const double* E, const double* Ubra, const double* Uket,
                    const SiteOp& w, int RB, double* out, const MixQ* q = nullptr);
  void env_right_raw(int rb, int rk, int rb2, int rk2, int RB, const double* E, const double* Ubra,
                     const double* Uket, const SiteOp& w, int RA, double* out, const MixQ* q = nullptr);
  void heff_grad_raw(int rl, int rr, int RA, int RB, int RC, const double* Lenv, const double* Renv,
                     const std::vector<int>& A1, const std::vector<int>& B1, const std::vector<double>& o1,
                     const std::vector<int>& A2, const std::vector<int>& B2, const std::vector<double>& o2,
                     const double* x, double* E, double* gx, double* gL, double* gR, std::vector<double>& gop1,
                     std::vector<double>& gop2);
  void mpo_grad(double* E, double* const* gops);
  // window operator of the MPO at sites (b, b+1) applied with caller environments
  void window_apply(int b, int rl, int rr, const int32_t* ql, const int32_t* qr, const double* Lenv,
                    const double* Renv, int prec, const double* x, double* y);

  // environment updates through a site of the MPO (handles coefficient blocks)
  void env_left(const Env& in, const Core& bra, const Core& ket, int site, Env& out);
  void env_right(const Env& in, const Core& bra, const Core& ket, int site, Env& out);
  void env_unit(Env& e, int R);
  double env_close(const Env& Lb, const Env& Rb);  // full contraction at one bond
  double overlap_chain(const std::vector<const Core*>& bra, const std::vector<const Core*>& ket);

  static void build_siteop(SiteOp& so, int nout, const std::vector<int>& out_idx, const std::vector<int>& in_idx,
                           const std::vector<double>& ops, hipStream_t s);

  // workspace
  DevMem ws0, ws1, ws2, ws3, wsd, wsp;
  DevMem dav_V, dav_AV, dav_t, dav_u, dav_Au, dav_c, dav_mask, dav_t2, dav_t3;
  DevMem dav_xd, dav_yd, dav_dc;  // dense product input/output, compressed diagonal
  DevMem dav_uk, dav_tk;          // several roots: their Ritz vectors, a residual
  DevMem wlow_x, wlow_y, wlow_L, wlow_R, wlow_Rt;
  DevMem envq_o, envq_i;  // charge arrays of the environment-update mix
  // block-sparse product workspaces (T1, T2, stage-4 panels, split-K partials)
  DevMem bs_t1, bs_t2, bs_t3, bs_part, bs_tmp;
  DevMem bs_x16;  // x in bfloat16 for the bf16 products with both operators precontracted
  DevMem bs_gg1[4], bs_gg2[4];  // heavy-row GEMM descriptors per row bucket (16, 32, 64, larger)
  DevMem be_t1, be_panel, be_up, be_tmp;  // block-sparse environment-update workspaces
  long long bs_zero_serial = -1;  // plan whose never-written T1 entries are zero in bs_t1
  // plan (serial, precision, workspace addresses) whose heavy-row GEMM descriptors bs_gg1/2 hold
  long long bs_gg_serial = -1;
  int bs_gg_prec = -1;
  const void* bs_gg_ptr[3] = {nullptr, nullptr, nullptr};
  int bs_zero_prec = -1;

  // releases every workspace buffer of this engine (a worker that ran out of device memory)
  void release_workspaces();
  // concurrent task limit learned from a device allocation failure (0: none)
  int oom_cap = 0;

 private:
  void free_caches();
};

// The entries of one sparse MPO core grouped by output channel (CSR on the host):
// ptr[nout + 1], src[nnz] (input channel), op64/op32[nnz][16]; at least one slot each.
void siteop_csr(int nout, const std::vector<int>& out_idx, const std::vector<int>& in_idx,
                const std::vector<double>& ops, std::vector<int>& ptr, std::vector<int>& src,
                std::vector<double>& op64, std::vector<float>& op32);
// The dense two-site product on raw operands, tables and workspaces (engine.cpp).
template <class T>
void heff_dense(Engine& E, int rl, int rr, int RA, const T* Lv, int RB, const int* p1, const int* s1, const T* o1,
                int RC, const int* p2, const int* s2, const T* o2, const T* Rv, const T* x, T* y, T* ws_a, T* ws_b,
                const T* Rtil, int P0, int nP, const WinTabs* tabs, bool timed);
// Device address of the fixed scratch array of the no-allocation entry point on `device`
// (looked up once per device, with that device current; noalloc.hip).
void* noalloc_scratch(int device);
constexpr size_t kNoallocScratchBytes = size_t(256) << 20;

void upload(DevMem& m, const void* h, size_t bytes, hipStream_t s);
void download(void* h, const DevMem& m, size_t bytes, hipStream_t s);

}  // namespace tt
