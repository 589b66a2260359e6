// HIP kernels for gfx950 (CDNA4): MFMA GEMM tiles, sparse MPO mixing and the
// bandwidth-bound vector operations of the Davidson solver.
#include "kernels.h"

#include <algorithm>
#include <cstdio>
#include <stdexcept>

namespace tt {

#define HIPCHECK(x)                                                                  \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) throw tt::HipError(std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// MFMA GEMM: 128x128 output tile per workgroup (4 waves of 64x64), K step 16.
// One 16x16x4 MFMA per (16x16 sub-tile, 4-deep K slice); lane l supplies
// A[l%16][l/16] and B[l/16][l%16].  Accumulator register v of lane l holds
// D[4*(l/16)+v][l%16] for FP32 and D[4*v+l/16][l%16] for FP64.
// ---------------------------------------------------------------------------
constexpr int BM = 128, BN = 128, BK = 16;

template <typename T>
__device__ inline void mfma_step(T a, T b, T (&acc)[4]);

template <>
__device__ inline void mfma_step<double>(double a, double b, double (&acc)[4]) {
  d4 c = {acc[0], acc[1], acc[2], acc[3]};
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  acc[0] = c[0]; acc[1] = c[1]; acc[2] = c[2]; acc[3] = c[3];
}

template <>
__device__ inline void mfma_step<float>(float a, float b, float (&acc)[4]) {
  f4 c = {acc[0], acc[1], acc[2], acc[3]};
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  acc[0] = c[0]; acc[1] = c[1]; acc[2] = c[2]; acc[3] = c[3];
}

template <typename T>
__device__ inline int acc_row(int lane, int v);
template <>
__device__ inline int acc_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <>
__device__ inline int acc_row<double>(int lane, int v) { return 4 * v + (lane >> 4); }

// Software-pipelined tile loop: the next K tile is fetched from global memory
// into registers while the MFMAs of the current tile run out of one of two
// LDS buffers.  Global loads move runs of RUN consecutive elements along the
// contiguous direction of each operand (16-byte vector loads when VEC).
template <typename T>
struct GemmCfg {
  static constexpr int BK = sizeof(T) == 4 ? 32 : 16;
  static constexpr int RUN = BM * BK / 256;  // elements per thread per operand tile
};

// Iterates the K tiles (start indices, multiples of BKT inside a segment) that
// a workgroup has to process, following the structural-zero tables.
template <int BKT>
struct KIter {
  const GemmArgs& g;
  int seg = 0, nseg = 1, mt, nt, bz;
  bool empty = false;
  __device__ KIter(const GemmArgs& g_, int mt_, int nt_, int bz_) : g(g_), mt(mt_), nt(nt_), bz(bz_) {
    if (g.skip && g.skip[((long long)bz * g.mtiles + mt) * g.ntiles + nt]) empty = true;
    if (g.kmode == 2) nseg = g.nkb;
  }
  __device__ void bounds(int s, int& lo, int& hi) const {
    if (g.kmode == 0) { lo = 0; hi = g.K; }
    else if (g.kmode == 1) {
      const int* t = g.ktab + ((long long)bz * g.mtiles + mt) * 2;
      lo = t[0]; hi = t[1];
    } else {
      const int* t = g.ktab + ((long long)nt * g.nkb + s) * 2;
      lo = s * g.kin + t[0]; hi = s * g.kin + t[1];
    }
    if (hi > g.K) hi = g.K;
    lo = (lo / BKT) * BKT;  // tiles start on the BKT grid (inner blocks are multiples of BKT)
  }
  __device__ int start_from(int s) {
    for (; s < nseg; ++s) {
      int lo, hi;
      bounds(s, lo, hi);
      if (lo < hi) { seg = s; return lo; }
    }
    return -1;
  }
  __device__ int first() { return empty ? -1 : start_from(0); }
  __device__ int next(int k0) {
    int lo, hi;
    bounds(seg, lo, hi);
    if (k0 + BKT < hi) return k0 + BKT;
    return start_from(seg + 1);
  }
};

template <typename T, bool VEC>
__device__ inline void load_run(const T* __restrict__ p, long long stride, bool full, int nvalid, T* r) {
  constexpr int RUN = GemmCfg<T>::RUN;
  if (VEC && full && stride == 1) {
    if constexpr (sizeof(T) == 4) {
      const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
      for (int u = 0; u < RUN / 4; ++u) {
        float4 v = q[u];
        r[4 * u] = v.x; r[4 * u + 1] = v.y; r[4 * u + 2] = v.z; r[4 * u + 3] = v.w;
      }
    } else {
      const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
      for (int u = 0; u < RUN / 2; ++u) {
        double2 v = q[u];
        r[2 * u] = v.x; r[2 * u + 1] = v.y;
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < RUN; ++u) r[u] = (u < nvalid) ? p[u * stride] : T(0);
  }
}

template <typename T, bool AK, bool BNC, bool VEC>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, const T* __restrict__ A, const T* __restrict__ B,
                                          T* __restrict__ C, const int mtile, const int ntile, const int bz) {
  constexpr int BKc = GemmCfg<T>::BK;
  constexpr int RUN = GemmCfg<T>::RUN;
  __shared__ T As[2][BKc][BM + 4];
  __shared__ T Bs[2][BKc][BN + 4];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = mtile * BM;
  const int n0 = ntile * BN;
    const T* Ab = A + (long long)bz * g.sAb;
  const T* Bb = B + (long long)bz * g.sBb;
  T* Cb = C + (long long)bz * g.sCb;

  // thread -> run assignment
  // k-contiguous operand: row = tid/2, k offset = (tid%2)*RUN
  // m/n-contiguous operand: k = tid/(BM/RUN), offset = (tid%(BM/RUN))*RUN
  constexpr int TPR = BM / RUN;
  const int kc_row = tid >> 1, kc_k = (tid & 1) * RUN;
  const int mc_k = tid / TPR, mc_off = (tid % TPR) * RUN;

  T ra[RUN], rb[RUN];
  auto fetch = [&](int k0) {
    if (AK) {
      const int gm = m0 + kc_row;
      const int kk = k0 + kc_k;
      const int nv = (gm < g.M) ? max(0, min(RUN, g.K - kk)) : 0;
      const T* p = Ab + (long long)gm * g.sAm + (long long)(kk / g.kin) * g.sAkb + (long long)(kk % g.kin) * g.sAkk;
      load_run<T, VEC>(nv > 0 ? p : Ab, g.sAkk, nv == RUN, nv, ra);
    } else {
      const int kk = k0 + mc_k;
      const int gm = m0 + mc_off;
      const int nv = (kk < g.K) ? max(0, min(RUN, g.M - gm)) : 0;
      const T* p = Ab + (long long)gm * g.sAm + (long long)(kk / g.kin) * g.sAkb + (long long)(kk % g.kin) * g.sAkk;
      load_run<T, VEC>(nv > 0 ? p : Ab, g.sAm, nv == RUN, nv, ra);
    }
    if (BNC) {
      const int kk = k0 + mc_k;
      const int gn = n0 + mc_off;
      const int nv = (kk < g.K) ? max(0, min(RUN, g.N - gn)) : 0;
      const T* p = Bb + (long long)(kk / g.kin) * g.sBkb + (long long)(kk % g.kin) * g.sBkk + (long long)gn * g.sBn;
      load_run<T, VEC>(nv > 0 ? p : Bb, g.sBn, nv == RUN, nv, rb);
    } else {
      const int gn = n0 + kc_row;
      const int kk = k0 + kc_k;
      const int nv = (gn < g.N) ? max(0, min(RUN, g.K - kk)) : 0;
      const T* p = Bb + (long long)(kk / g.kin) * g.sBkb + (long long)(kk % g.kin) * g.sBkk + (long long)gn * g.sBn;
      load_run<T, VEC>(nv > 0 ? p : Bb, g.sBkk, nv == RUN, nv, rb);
    }
  };
  auto stash = [&](int buf) {
    if (AK) {
#pragma unroll
      for (int u = 0; u < RUN; ++u) As[buf][kc_k + u][kc_row] = ra[u];
    } else {
#pragma unroll
      for (int u = 0; u < RUN; ++u) As[buf][mc_k][mc_off + u] = ra[u];
    }
    if (BNC) {
#pragma unroll
      for (int u = 0; u < RUN; ++u) Bs[buf][mc_k][mc_off + u] = rb[u];
    } else {
#pragma unroll
      for (int u = 0; u < RUN; ++u) Bs[buf][kc_k + u][kc_row] = rb[u];
    }
  };

  T acc[4][4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);

  KIter<BKc> it(g, mtile, ntile, bz);
  int buf = 0;
  int kcur = it.first();
  if (kcur >= 0) {
    fetch(kcur);
    stash(0);
  }
  __syncthreads();
  while (kcur >= 0) {
    const int knext = it.next(kcur);
    const bool more = knext >= 0;
    if (more) fetch(knext);
#pragma unroll
    for (int ks = 0; ks < BKc; ks += 4) {
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][ks + (lane >> 4)][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[buf][ks + (lane >> 4)][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) mfma_step<T>(a[i], b[j], acc[i][j]);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    kcur = knext;
  }
  // ---- epilogue ----
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn * 64 + j * 16 + (lane & 15);
      if (col >= g.N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 64 + i * 16 + acc_row<T>(lane, v);
        if (row >= g.M) continue;
        T* p = Cb + (long long)row * g.sCm + col;
        T r = T(g.alpha) * acc[i][j][v];
        if (g.beta != 0.0) r += T(g.beta) * (*p);
        *p = r;
      }
    }
}

template <typename T, bool AK, bool BNC, bool VEC>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g, const T* __restrict__ A, const T* __restrict__ B,
                                                   T* __restrict__ C) {
  gemm_tile<T, AK, BNC, VEC>(g, A, B, C, blockIdx.x, blockIdx.y, blockIdx.z);
}

// one launch for a list of independent GEMMs: blockIdx.z selects the problem,
// tiles outside it return at once
template <typename T, bool AK, bool BNC, bool VEC>
__global__ __launch_bounds__(256) void gemm_grouped_kernel(const GemmGroup<T>* __restrict__ grp) {
  const GemmGroup<T> G = grp[blockIdx.z];
  if ((int)blockIdx.x * BM >= G.g.M || (int)blockIdx.y * BN >= G.g.N) return;
  gemm_tile<T, AK, BNC, VEC>(G.g, G.A, G.B, G.C, blockIdx.x, blockIdx.y, 0);
}

static void check_args(const GemmArgs& g) {
  if (g.M < 0 || g.N < 0 || g.K < 0 || g.batch < 0) throw std::runtime_error("gemm: negative size");
  if (g.kin <= 0 || g.kin % BK != 0) throw std::runtime_error("gemm: inner K block must be a multiple of 16");
}

template <typename T>
void gemm(const GemmArgs& g, const T* A, const T* B, T* C, bool a_kcontig, bool b_ncontig, hipStream_t s) {
  check_args(g);
  if (g.M == 0 || g.N == 0 || g.batch == 0) return;
  if (!C || (g.K > 0 && (!A || !B))) throw std::runtime_error("gemm: null operand");
  if (g.K == 0) {
    // C = beta*C : run the kernel anyway (loop body skipped) for uniform semantics
  }
  dim3 grid((g.M + BM - 1) / BM, (g.N + BN - 1) / BN, g.batch);
  if (grid.y > 65535 || grid.z > 65535) throw std::runtime_error("gemm: grid too large");
  // 16-byte vector loads need every stride that moves a run start, and the base
  // pointers, to be aligned to 16 bytes
  constexpr long long VW = 16 / sizeof(T);
  const bool vec = ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) && g.sAb % VW == 0 && g.sBb % VW == 0 &&
                   g.sAkb % VW == 0 && g.sBkb % VW == 0 && (a_kcontig ? g.sAm % VW == 0 : g.sAkk % VW == 0) &&
                   (b_ncontig ? g.sBkk % VW == 0 : g.sBn % VW == 0) && g.kin % GemmCfg<T>::RUN == 0;
#define LAUNCH(AKc, BNc, V) \
  hipLaunchKernelGGL((gemm_kernel<T, AKc, BNc, V>), grid, dim3(256), 0, s, g, A, B, C)
  if (vec) {
    if (a_kcontig && b_ncontig) LAUNCH(true, true, true);
    else if (a_kcontig) LAUNCH(true, false, true);
    else if (b_ncontig) LAUNCH(false, true, true);
    else LAUNCH(false, false, true);
  } else {
    if (a_kcontig && b_ncontig) LAUNCH(true, true, false);
    else if (a_kcontig) LAUNCH(true, false, false);
    else if (b_ncontig) LAUNCH(false, true, false);
    else LAUNCH(false, false, false);
  }
#undef LAUNCH
  HIPCHECK(hipGetLastError());
}

template <typename T>
void gemm_grouped(const GemmGroup<T>* dev_groups, const std::vector<GemmGroup<T>>& host_groups, hipStream_t s) {
  if (host_groups.empty()) return;
  constexpr long long VW = 16 / sizeof(T);
  int mt = 0, nt = 0;
  bool vec = true;
  for (const GemmGroup<T>& G : host_groups) {
    const GemmArgs& g = G.g;
    check_args(g);
    if (g.batch != 1) throw std::runtime_error("gemm_grouped: one batch per problem");
    if (g.kmode != 0 || g.skip) throw std::runtime_error("gemm_grouped: dense problems only");
    if (g.M > 0 && g.N > 0 && g.K > 0 && (!G.A || !G.B || !G.C)) throw std::runtime_error("gemm_grouped: null operand");
    mt = std::max(mt, (g.M + BM - 1) / BM);
    nt = std::max(nt, (g.N + BN - 1) / BN);
    vec = vec && ((uintptr_t)G.A % 16 == 0) && ((uintptr_t)G.B % 16 == 0) && g.sAm % VW == 0 && g.sBkk % VW == 0 &&
          g.kin % GemmCfg<T>::RUN == 0 && g.sAkk == 1 && g.sBn == 1;
    if (g.sAkk != 1 || g.sBn != 1) throw std::runtime_error("gemm_grouped: row-major operands only");
  }
  if (mt == 0 || nt == 0) return;
  if (nt > 65535 || host_groups.size() > 65535) throw std::runtime_error("gemm_grouped: grid too large");
  dim3 grid(mt, nt, (unsigned)host_groups.size());
  if (vec)
    hipLaunchKernelGGL((gemm_grouped_kernel<T, true, true, true>), grid, dim3(256), 0, s, dev_groups);
  else
    hipLaunchKernelGGL((gemm_grouped_kernel<T, true, true, false>), grid, dim3(256), 0, s, dev_groups);
  HIPCHECK(hipGetLastError());
}
// ---------------------------------------------------------------------------
// skinny grouped GEMM: C[m][n] = sum_k A[m][k] B[k][n] for M <= 64 rows
// ---------------------------------------------------------------------------
template <typename T, int MB>
__global__ __launch_bounds__(256) void skinny_mfma_kernel(const GemmGroup<T>* __restrict__ grp) {
  constexpr int KS = sizeof(T) == 4 ? 16 : 8;  // K slice
  constexpr int NB = 256;                      // columns per workgroup
  constexpr int MRW = MB * 16;
  constexpr int BPT = KS * NB / 256;           // B elements per thread per slice
  __shared__ T As[2][KS][MRW + 4];
  __shared__ T Bs[2][KS][NB + 4];
  const GemmGroup<T> G = grp[blockIdx.y];
  const int M = G.g.M, N = G.g.N, K = G.g.K;
  const long long lda = G.g.sAm, ldb = G.g.sBkk, ldc = G.g.sCm;
  const int n0 = (int)blockIdx.x * NB;
  if (n0 >= N) return;  // uniform over the workgroup
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // B: thread -> row br, BPT consecutive columns from bc
  constexpr int TPR = NB / BPT;  // threads per B row
  const int br = tid / TPR, bc = (tid % TPR) * BPT;
  const bool bvec = ((ldb * sizeof(T)) % 16 == 0) && ((reinterpret_cast<uintptr_t>(G.B) % 16) == 0);
  T rb[BPT];
  constexpr int AP = (MRW * KS + 255) / 256;  // A elements per thread per slice
  T ra[AP];
  auto fetch = [&](int k0) {
    const int k = k0 + br;
    const long long base = (long long)k * ldb + n0 + bc;
    if (k < K && bvec && n0 + bc + BPT <= N) {
#pragma unroll
      for (int u = 0; u < BPT; u += 16 / (int)sizeof(T)) {
        if constexpr (sizeof(T) == 4) {
          const float4 v = *reinterpret_cast<const float4*>(G.B + base + u);
          rb[u] = v.x; rb[u + 1] = v.y; rb[u + 2] = v.z; rb[u + 3] = v.w;
        } else {
          const double2 v = *reinterpret_cast<const double2*>(G.B + base + u);
          rb[u] = v.x; rb[u + 1] = v.y;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < BPT; ++u) rb[u] = (k < K && n0 + bc + u < N) ? G.B[base + u] : T(0);
    }
#pragma unroll
    for (int u = 0; u < AP; ++u) {
      const int e = tid + u * 256, ar = e / KS, ak = e - ar * KS;
      ra[u] = (e < MRW * KS && ar < M && k0 + ak < K) ? G.A[(long long)ar * lda + k0 + ak] : T(0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < BPT; ++u) Bs[buf][br][bc + u] = rb[u];
#pragma unroll
    for (int u = 0; u < AP; ++u) {
      const int e = tid + u * 256, ar = e / KS, ak = e - ar * KS;
      if (e < MRW * KS) As[buf][ak][ar] = ra[u];
    }
  };
  T acc[MB][4][4];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);
  int buf = 0;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int k0 = 0; k0 < K; k0 += KS) {
    const bool more = k0 + KS < K;
    if (more) fetch(k0 + KS);
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      T b[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[buf][kk + (lane >> 4)][wv * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        const T a = As[buf][kk + (lane >> 4)][i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 4; ++j) mfma_step<T>(a, b[j], acc[i][j]);
      }
    }
    if (more) {
      // buf ^ 1 was last read before the previous barrier
      stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wv * 64 + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i * 16 + acc_row<T>(lane, v);
        if (row < M) G.C[(long long)row * ldc + col] = acc[i][j][v];
      }
    }
}

int skinny_rows(int M) {
  if (M <= 0) return 16;
  if (M > kSkinnyMaxM) return 0;
  return (M + 15) / 16 * 16;
}

template <typename T>
void gemm_grouped_skinny(const GemmGroup<T>* dev_groups, const std::vector<GemmGroup<T>>& host_groups, int mr,
                         hipStream_t s) {
  if (host_groups.empty()) return;
  int nmax = 0;
  for (const GemmGroup<T>& G : host_groups) {
    const GemmArgs& g = G.g;
    check_args(g);
    if (g.batch != 1 || g.kmode != 0 || g.skip) throw std::runtime_error("gemm_grouped_skinny: dense problems only");
    if (g.M > mr) throw std::runtime_error("gemm_grouped_skinny: more rows than the bucket");
    if (g.sAkk != 1 || g.sBn != 1) throw std::runtime_error("gemm_grouped_skinny: row-major operands only");
    if (g.alpha != 1.0 || g.beta != 0.0) throw std::runtime_error("gemm_grouped_skinny: C = A B only");
    if (g.K > g.kin) throw std::runtime_error("gemm_grouped_skinny: one inner K block only");
    if (g.M > 0 && g.N > 0 && g.K > 0 && (!G.A || !G.B || !G.C)) throw std::runtime_error("gemm_grouped_skinny: null operand");
    nmax = std::max(nmax, g.N);
  }
  if (nmax == 0) return;
  dim3 grid((nmax + 255) / 256, (unsigned)host_groups.size(), 1);
  if (grid.y > 65535) throw std::runtime_error("gemm_grouped_skinny: too many problems");
  if (mr == 16) hipLaunchKernelGGL((skinny_mfma_kernel<T, 1>), grid, dim3(256), 0, s, dev_groups);
  else if (mr == 32) hipLaunchKernelGGL((skinny_mfma_kernel<T, 2>), grid, dim3(256), 0, s, dev_groups);
  else if (mr == 48) hipLaunchKernelGGL((skinny_mfma_kernel<T, 3>), grid, dim3(256), 0, s, dev_groups);
  else if (mr == 64) hipLaunchKernelGGL((skinny_mfma_kernel<T, 4>), grid, dim3(256), 0, s, dev_groups);
  else throw std::runtime_error("gemm_grouped_skinny: row bucket must be 16, 32, 48 or 64");
  HIPCHECK(hipGetLastError());
}
template void gemm_grouped_skinny<double>(const GemmGroup<double>*, const std::vector<GemmGroup<double>>&, int,
                                          hipStream_t);
template void gemm_grouped_skinny<float>(const GemmGroup<float>*, const std::vector<GemmGroup<float>>&, int,
                                         hipStream_t);

template void gemm_grouped<double>(const GemmGroup<double>*, const std::vector<GemmGroup<double>>&, hipStream_t);
template void gemm_grouped<float>(const GemmGroup<float>*, const std::vector<GemmGroup<float>>&, hipStream_t);

template void gemm<double>(const GemmArgs&, const double*, const double*, double*, bool, bool, hipStream_t);
template void gemm<float>(const GemmArgs&, const float*, const float*, float*, bool, bool, hipStream_t);

// ---------------------------------------------------------------------------
// BF16 operands, FP32 accumulation: 16x16x32 MFMA (gfx950).  Lane l supplies
// A[l%16][8*(l/16)+0..7] and B[8*(l/16)+0..7][l%16].  K step 32.
// ---------------------------------------------------------------------------
constexpr int BK16 = 32;

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <bool AK, bool BNC>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g, const uint16_t* __restrict__ A,
                                                        const uint16_t* __restrict__ B, float* __restrict__ C) {
  __shared__ uint16_t As[BM][BK16 + 8];  // [m][k]
  __shared__ uint16_t Bs[BN][BK16 + 8];  // [n][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const int bz = blockIdx.z;
  const uint16_t* Ab = A + (long long)bz * g.sAb;
  const uint16_t* Bb = B + (long long)bz * g.sBb;
  float* Cb = C + (long long)bz * g.sCb;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  KIter<BK16> it(g, blockIdx.x, blockIdx.y, bz);
  for (int k0 = it.first(); k0 >= 0; k0 = it.next(k0)) {
    const long long kbase_a = (long long)(k0 / g.kin) * g.sAkb;
    const long long kbase_b = (long long)(k0 / g.kin) * g.sBkb;
    const int kr = k0 % g.kin;
    // A tile: 128 x 32 = 4096 elements, 16 per thread
    if (AK) {
      const int m = tid >> 1, kh = (tid & 1) * 16;
      const int gm = m0 + m;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int kk = kh + u;
        uint16_t v = 0;
        if (gm < g.M && k0 + kk < g.K) v = Ab[(long long)gm * g.sAm + kbase_a + (long long)(kr + kk) * g.sAkk];
        As[m][kk] = v;
      }
    } else {
      const int kk = tid >> 3, mc = (tid & 7) * 16;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int gm = m0 + mc + u;
        uint16_t v = 0;
        if (gm < g.M && k0 + kk < g.K) v = Ab[(long long)gm * g.sAm + kbase_a + (long long)(kr + kk) * g.sAkk];
        As[mc + u][kk] = v;
      }
    }
    if (BNC) {
      const int kk = tid >> 3, nc = (tid & 7) * 16;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int gn = n0 + nc + u;
        uint16_t v = 0;
        if (gn < g.N && k0 + kk < g.K) v = Bb[kbase_b + (long long)(kr + kk) * g.sBkk + (long long)gn * g.sBn];
        Bs[nc + u][kk] = v;
      }
    } else {
      const int n = tid >> 1, kh = (tid & 1) * 16;
      const int gn = n0 + n;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int kk = kh + u;
        uint16_t v = 0;
        if (gn < g.N && k0 + kk < g.K) v = Bb[kbase_b + (long long)(kr + kk) * g.sBkk + (long long)gn * g.sBn];
        Bs[n][kk] = v;
      }
    }
    __syncthreads();
    bf8 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint16_t* p = &As[wm * 64 + i * 16 + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[i][u] = __builtin_bit_cast(__bf16, p[u]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint16_t* p = &Bs[wn * 64 + j * 16 + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[j][u] = __builtin_bit_cast(__bf16, p[u]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn * 64 + j * 16 + (lane & 15);
      if (col >= g.N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        if (row >= g.M) continue;
        float* p = Cb + (long long)row * g.sCm + col;
        float r = (float)g.alpha * acc[i][j][v];
        if (g.beta != 0.0) r += (float)g.beta * (*p);
        *p = r;
      }
    }
}

void gemm_bf16(const GemmArgs& g, const uint16_t* A, const uint16_t* B, float* C, bool a_kcontig, bool b_ncontig,
               hipStream_t s) {
  if (g.kin <= 0 || g.kin % BK16 != 0) throw std::runtime_error("gemm_bf16: inner K block must be a multiple of 32");
  if (g.M == 0 || g.N == 0 || g.batch == 0) return;
  if (!C || (g.K > 0 && (!A || !B))) throw std::runtime_error("gemm: null operand");
  dim3 grid((g.M + BM - 1) / BM, (g.N + BN - 1) / BN, g.batch);
  if (grid.y > 65535 || grid.z > 65535) throw std::runtime_error("gemm: grid too large");
  if (a_kcontig && b_ncontig)
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(256), 0, s, g, A, B, C);
  else if (a_kcontig && !b_ncontig)
    hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(256), 0, s, g, A, B, C);
  else if (!a_kcontig && b_ncontig)
    hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(256), 0, s, g, A, B, C);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(256), 0, s, g, A, B, C);
  HIPCHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Sparse MPO mixing (memory bound).  One wave per (output channel, chunk of 64
// positions).  Workgroups are dispatched round-robin over the 8 XCDs, so the
// linear workgroup id is mapped such that XCD x owns the chunks c = x mod 8 and
// walks through every output channel of one chunk before the next: the input
// slabs of that chunk (all channels, 64 positions x 4 states) stay resident in
// the XCD's own L2 while the fan-in gathers re-read them.
// ---------------------------------------------------------------------------
constexpr int MIX_CHUNK = 64;
constexpr int NXCD = 8;

__device__ inline bool site_charge(int dn, int ds) {
  return (dn == 0 && ds == 0) || (dn == 1 && (ds == 1 || ds == -1)) || (dn == 2 && ds == 0);
}

template <typename T>
__global__ __launch_bounds__(MIX_CHUNK) void mix_kernel(const int* __restrict__ ptr, const int* __restrict__ src,
                                                        const T* __restrict__ op, const T* __restrict__ in,
                                                        long long in_cs, T* __restrict__ out, long long out_cs,
                                                        int O, int I, int nout, long long nchunks, MixQ q) {
  const long long w = blockIdx.x;
  const long long xcd = w % NXCD;
  const long long j = w / NXCD;
  const long long c = (j / nout) * NXCD + xcd;  // chunk owned by this XCD
  const int ch = (int)(j % nout);
  if (c >= nchunks) return;
  const long long p = c * MIX_CHUNK + threadIdx.x;
  const long long npos = (long long)O * I;
  if (p >= npos) return;
  const long long o = p / I, i = p % I;
  const long long off = o * 4LL * I + i;
  T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  bool live = true;
  if (q.qo) {
    const int2 a = q.qo[o], b = q.qi[i], cc = q.qc[ch];
    live = site_charge(b.x - a.x + q.sgn * cc.x, b.y - a.y + q.sgn * cc.y);
  }
  if (live) {
    const int e0 = ptr[ch], e1 = ptr[ch + 1];
    for (int e = e0; e < e1; ++e) {
      const T* wt = op + 16LL * e;
      const T* x = in + (long long)src[e] * in_cs + off;
      const T v0 = x[0], v1 = x[I], v2 = x[2LL * I], v3 = x[3LL * I];
      acc0 += wt[0] * v0 + wt[1] * v1 + wt[2] * v2 + wt[3] * v3;
      acc1 += wt[4] * v0 + wt[5] * v1 + wt[6] * v2 + wt[7] * v3;
      acc2 += wt[8] * v0 + wt[9] * v1 + wt[10] * v2 + wt[11] * v3;
      acc3 += wt[12] * v0 + wt[13] * v1 + wt[14] * v2 + wt[15] * v3;
    }
  }
  T* y = out + (long long)ch * out_cs + off;
  y[0] = acc0;
  y[I] = acc1;
  y[2LL * I] = acc2;
  y[3LL * I] = acc3;
}

template <typename T>
void mix(int nout, const int* ptr, const int* src, const T* op, const T* in, long long in_cs, T* out,
         long long out_cs, int O, int I, hipStream_t s, const MixQ* q) {
  if (nout == 0 || O == 0 || I == 0) return;
  if (!ptr || !src || !op || !in || !out) throw std::runtime_error("mix: null operand");
  const long long npos = (long long)O * I;
  const long long nchunks = (npos + MIX_CHUNK - 1) / MIX_CHUNK;
  const long long nchunks_pad = ((nchunks + NXCD - 1) / NXCD) * NXCD;
  const long long nblk = nchunks_pad * nout;
  if (nblk > 2147483647LL) throw std::runtime_error("mix: grid too large");
  MixQ qq;
  if (q && q->qo && q->qi && q->qc) qq = *q;
  hipLaunchKernelGGL((mix_kernel<T>), dim3((unsigned)nblk), dim3(MIX_CHUNK), 0, s, ptr, src, op, in, in_cs, out,
                     out_cs, O, I, nout, nchunks, qq);
  HIPCHECK(hipGetLastError());
}

template void mix<double>(int, const int*, const int*, const double*, const double*, long long, double*, long long,
                          int, int, hipStream_t, const MixQ*);
template void mix<float>(int, const int*, const int*, const float*, const float*, long long, float*, long long, int,
                         int, hipStream_t, const MixQ*);

// ---------------------------------------------------------------------------
// vector kernels
// ---------------------------------------------------------------------------
static inline unsigned nblocks(size_t n, int per = 256) {
  size_t b = (n + per - 1) / per;
  return (unsigned)std::min<size_t>(b, 1u << 20);
}

__global__ void fill_kernel(uint32_t* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}
__global__ void fill8_kernel(uint8_t* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

void fill(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (bytes % 4 == 0 && ((uintptr_t)p % 4) == 0)
    hipLaunchKernelGGL(fill_kernel, dim3(nblocks(bytes / 4)), dim3(256), 0, s, (uint32_t*)p, bytes / 4);
  else
    hipLaunchKernelGGL(fill8_kernel, dim3(nblocks(bytes)), dim3(256), 0, s, (uint8_t*)p, bytes);
  HIPCHECK(hipGetLastError());
}

__global__ void scale_kernel(double* x, double a, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) x[i] *= a;
}
void scale(double* x, double a, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(scale_kernel, dim3(nblocks(n)), dim3(256), 0, s, x, a, n);
  HIPCHECK(hipGetLastError());
}

__global__ void axpy_kernel(double* y, double a, const double* x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}
void axpy(double* y, double a, const double* x, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(axpy_kernel, dim3(nblocks(n)), dim3(256), 0, s, y, a, x, n);
  HIPCHECK(hipGetLastError());
}

__global__ void axpby_kernel(double* z, double a, const double* x, double b, const double* y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    z[i] = a * x[i] + b * y[i];
}
void axpby(double* z, double a, const double* x, double b, const double* y, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(256), 0, s, z, a, x, b, y, n);
  HIPCHECK(hipGetLastError());
}

__global__ void mask_kernel(double* x, const uint8_t* m, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!m[i]) x[i] = 0.0;
}
void mask_apply(double* x, const uint8_t* mask, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(mask_kernel, dim3(nblocks(n)), dim3(256), 0, s, x, mask, n);
  HIPCHECK(hipGetLastError());
}

// compressed vector <-> dense tensor through an index list of the kept entries
__global__ void gather_idx_kernel(double* out, const double* in, const int* idx, size_t nc, size_t ncp) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ncp; i += (size_t)gridDim.x * blockDim.x)
    out[i] = i < nc ? in[idx[i]] : 0.0;
}
__global__ void scatter_idx_kernel(double* out, const double* in, const int* idx, size_t nc) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nc; i += (size_t)gridDim.x * blockDim.x)
    out[idx[i]] = in[i];
}
void gather_idx(double* out, const double* in, const int* idx, size_t nc, size_t ncp, hipStream_t s) {
  if (!ncp) return;
  hipLaunchKernelGGL(gather_idx_kernel, dim3(nblocks(ncp)), dim3(256), 0, s, out, in, idx, nc, ncp);
  HIPCHECK(hipGetLastError());
}
void scatter_idx(double* out, const double* in, const int* idx, size_t nc, hipStream_t s) {
  if (!nc) return;
  hipLaunchKernelGGL(scatter_idx_kernel, dim3(nblocks(nc)), dim3(256), 0, s, out, in, idx, nc);
  HIPCHECK(hipGetLastError());
}

// Two-pass deterministic multi-dot.  First pass: partial[i][blk] = sum over the
// block's grid-stride share of V_i . w.  A block takes the vectors CNT <= 8 at a time
// (w is read once per pass); with VEC = 2 every load is 16 bytes.  Sums are reduced
// within each wave by butterfly shuffles, then over the block's four waves in a fixed
// order, so the result depends only on n and the number of blocks.
template <int CNT, int VEC>
__device__ __forceinline__ void mdot_pass(const double* __restrict__ V, size_t ldv, int i0,
                                          const double* __restrict__ w, size_t nv, int nblk, double (&s)[8]) {
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] = 0.0;
  for (size_t k = blockIdx.x * (size_t)256 + threadIdx.x; k < nv; k += (size_t)nblk * 256) {
    if constexpr (VEC == 2) {
      const double2 wk = reinterpret_cast<const double2*>(w)[k];
      double2 v[CNT];
#pragma unroll
      for (int u = 0; u < CNT; ++u) v[u] = reinterpret_cast<const double2*>(V + (size_t)(i0 + u) * ldv)[k];
#pragma unroll
      for (int u = 0; u < CNT; ++u) {
        s[u] = fma(v[u].x, wk.x, s[u]);
        s[u] = fma(v[u].y, wk.y, s[u]);
      }
    } else {
      const double wk = w[k];
      double v[CNT];
#pragma unroll
      for (int u = 0; u < CNT; ++u) v[u] = V[(size_t)(i0 + u) * ldv + k];
#pragma unroll
      for (int u = 0; u < CNT; ++u) s[u] = fma(v[u], wk, s[u]);
    }
  }
}
template <int VEC>
__global__ __launch_bounds__(256) void mdot_partial(const double* __restrict__ V, size_t ldv, int m,
                                                    const double* __restrict__ w, size_t n, double* __restrict__ partial,
                                                    int nblk) {
  __shared__ double red[4][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t nv = n / VEC;
  for (int i0 = 0; i0 < m; i0 += 8) {
    const int cnt = min(8, m - i0);
    double s[8];
    switch (cnt) {
      case 1: mdot_pass<1, VEC>(V, ldv, i0, w, nv, nblk, s); break;
      case 2: mdot_pass<2, VEC>(V, ldv, i0, w, nv, nblk, s); break;
      case 3: mdot_pass<3, VEC>(V, ldv, i0, w, nv, nblk, s); break;
      case 4: mdot_pass<4, VEC>(V, ldv, i0, w, nv, nblk, s); break;
      case 5: mdot_pass<5, VEC>(V, ldv, i0, w, nv, nblk, s); break;
      case 6: mdot_pass<6, VEC>(V, ldv, i0, w, nv, nblk, s); break;
      case 7: mdot_pass<7, VEC>(V, ldv, i0, w, nv, nblk, s); break;
      default: mdot_pass<8, VEC>(V, ldv, i0, w, nv, nblk, s); break;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      for (int o = 32; o > 0; o >>= 1) s[u] += __shfl_xor(s[u], o, 64);
    if (lane == 0)
#pragma unroll
      for (int u = 0; u < 8; ++u) red[wave][u] = s[u];
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const int u = threadIdx.x;
      partial[(size_t)(i0 + u) * nblk + blockIdx.x] = (red[0][u] + red[1][u]) + (red[2][u] + red[3][u]);
    }
    __syncthreads();
  }
}
// out[i] = sum_blk partial[i][blk], one block per output (fixed-order tree: deterministic)
__global__ __launch_bounds__(256) void mdot_final(const double* __restrict__ partial, int nblk,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(size_t)i * nblk + b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}
int dot_blocks(size_t n) {
  // at least 2048 elements (eight 16-byte loads per thread) per block, at most kDotBlocks
  return (int)std::min<size_t>(kDotBlocks, std::max<size_t>(1, (n + 2047) / 2048));
}
void multi_dot(const double* V, size_t ldv, int m, const double* w, size_t n, double* out_dev, double* partial,
               int cap_blk, hipStream_t s) {
  if (m <= 0) return;
  if (m > 65535) throw std::runtime_error("multi_dot: too many vectors");
  if (cap_blk <= 0) throw std::runtime_error("multi_dot: no partial-sum buffer");
  const int nblk = std::min(cap_blk, dot_blocks(n));
  const bool vec2 = n % 2 == 0 && ldv % 2 == 0 && (uintptr_t)V % 16 == 0 && (uintptr_t)w % 16 == 0;
  if (vec2)
    hipLaunchKernelGGL(mdot_partial<2>, dim3(nblk), dim3(256), 0, s, V, ldv, m, w, n, partial, nblk);
  else
    hipLaunchKernelGGL(mdot_partial<1>, dim3(nblk), dim3(256), 0, s, V, ldv, m, w, n, partial, nblk);
  HIPCHECK(hipGetLastError());
  hipLaunchKernelGGL(mdot_final, dim3(m), dim3(256), 0, s, partial, nblk, out_dev);
  HIPCHECK(hipGetLastError());
}

// One-sided (Hestenes) Jacobi SVD, one workgroup of JW waves per matrix.  Each sweep
// visits every column pair once in N' - 1 rounds of a round-robin tournament (N' = N
// rounded up to even; player N' - 1 stays, the others rotate), so the N'/2 pairs of a
// round are disjoint and the waves take them in turn.  A pair (p, q) is rotated when
// |a_p . a_q| > tol |a_p| |a_q| (tol = M eps) and neither column is numerically zero
// (|a|^2 <= tol^2 |A|_F^2: rotations with larger columns keep refilling such a column with
// rounding noise of its own size, so it never meets the relative test; its singular value
// lies far below any truncation cutoff).  The same rotation is applied to the columns of V,
// and columns of up to 64 JR rows stay in registers between the dot products and the
// rotation.
// After convergence sigma_j = |a_j|, u_j = a_j / sigma_j, and the triplets are written
// in decreasing order of sigma (ties by column index).  With INLDS the matrix and V are
// held in LDS for the whole factorisation ((M + N) N <= kJacobiLds doubles).
constexpr int JW = 16;  // waves per workgroup
constexpr int JR = 8;   // rows per lane held in registers (columns of up to 512 rows)
// Sum over the 64 lanes of a wave, the same value in every lane.  Within each row of 16
// lanes the partial sums are exchanged by DPP moves (xor 1 and xor 2 as quad permutations,
// then the half-row and row mirrors), each step adding two values that the exchanged lanes
// hold in swapped order, so all lanes of a row agree bit for bit; the four row sums are then
// read into scalars and added in a fixed order.  DPP moves stay in the register file, far
// cheaper than shuffles through the LDS crossbar.
template <int CTRL>
__device__ __forceinline__ double dpp_add(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return v + __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  v = dpp_add<0x141>(v);  // row_half_mirror: lane i <-> 7 - i within 8
  v = dpp_add<0x140>(v);  // row_mirror: lane i <-> 15 - i within 16
  auto row = [&](int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
  };
  return (row(0) + row(16)) + (row(32) + row(48));
}
template <bool INLDS>
__global__ __launch_bounds__(64 * JW) void jacobi_svd_kernel(const SvdJob* __restrict__ jobs, int max_sweeps) {
  __shared__ double sig[kJacobiMaxN];
  __shared__ int rnk[kJacobiMaxN];
  __shared__ int rotated;
  __shared__ double lds[INLDS ? kJacobiLds : 1];
  const SvdJob J = jobs[blockIdx.x];
  const int M = J.M, N = J.N, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NT = 64 * JW;
  if (N <= 0 || N > kJacobiMaxN || M < N || J.lda < M || J.ldu < M || J.ldvt < N ||
      (INLDS && (long long)(M + N) * N > kJacobiLds)) {
    if (tid == 0) J.info[0] = -1;
    return;
  }
  // column j of the working matrix starts at A + j * lda (compact in LDS)
  const int lda = INLDS ? M : J.lda;
  double* A = INLDS ? lds : J.A;
  double* V = INLDS ? lds + (size_t)M * N : J.V;
  if (INLDS)
    for (int i = tid; i < M * N; i += NT) A[i] = J.A[(size_t)(i / M) * J.lda + i % M];
  for (long long i = tid; i < (long long)N * N; i += NT) V[i] = (i % (N + 1) == 0) ? 1.0 : 0.0;
  __syncthreads();
  __shared__ double fro_w[JW];
  {
    double s2 = 0.0;
    for (int j = wave; j < N; j += JW)
      for (int i = lane; i < M; i += 64) s2 = fma(A[(size_t)j * lda + i], A[(size_t)j * lda + i], s2);
    s2 = wave_sum(s2);
    if (lane == 0) fro_w[wave] = s2;
  }
  __syncthreads();
  double fro2 = 0.0;
  for (int w = 0; w < JW; ++w) fro2 += fro_w[w];
  const double tol = 2.2e-16 * (double)M;
  const double zero2 = tol * tol * fro2;  // |a_j|^2 at or below this: a numerically zero column
  const int Np = N + (N & 1);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < Np - 1; ++r) {
      for (int k = wave; k < Np / 2; k += JW) {
        int p, q;
        if (k == 0) { p = Np - 1; q = r; }
        else { p = (r + k) % (Np - 1); q = (r - k + Np - 1) % (Np - 1); }
        if (p >= N || q >= N) continue;
        double* ap = A + (size_t)p * lda;
        double* aq = A + (size_t)q * lda;
        double al = 0.0, be = 0.0, ga = 0.0;
        if (M <= 64 * JR) {
          // both columns stay in registers between the dot products and the rotation
          double x[JR], y[JR];
#pragma unroll
          for (int u = 0; u < JR; ++u) {
            const int i = lane + 64 * u;
            x[u] = i < M ? ap[i] : 0.0;
            y[u] = i < M ? aq[i] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < JR; ++u) {
            al = fma(x[u], x[u], al);
            be = fma(y[u], y[u], be);
            ga = fma(x[u], y[u], ga);
          }
          al = wave_sum(al);
          be = wave_sum(be);
          ga = wave_sum(ga);
          if (!(fabs(ga) > tol * sqrt(al * be)) || !(fmin(al, be) > zero2)) continue;
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll
          for (int u = 0; u < JR; ++u) {
            const int i = lane + 64 * u;
            if (i < M) {
              ap[i] = c * x[u] - sn * y[u];
              aq[i] = sn * x[u] + c * y[u];
            }
          }
          double* vp = V + (size_t)p * N;
          double* vq = V + (size_t)q * N;
          for (int i = lane; i < N; i += 64) {
            const double xv = vp[i], yv = vq[i];
            vp[i] = c * xv - sn * yv;
            vq[i] = sn * xv + c * yv;
          }
        } else {
          for (int i = lane; i < M; i += 64) {
            const double x = ap[i], y = aq[i];
            al = fma(x, x, al);
            be = fma(y, y, be);
            ga = fma(x, y, ga);
          }
          al = wave_sum(al);
          be = wave_sum(be);
          ga = wave_sum(ga);
          if (!(fabs(ga) > tol * sqrt(al * be)) || !(fmin(al, be) > zero2)) continue;
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          for (int i = lane; i < M; i += 64) {
            const double x = ap[i], y = aq[i];
            ap[i] = c * x - sn * y;
            aq[i] = sn * x + c * y;
          }
          double* vp = V + (size_t)p * N;
          double* vq = V + (size_t)q * N;
          for (int i = lane; i < N; i += 64) {
            const double x = vp[i], y = vq[i];
            vp[i] = c * x - sn * y;
            vq[i] = sn * x + c * y;
          }
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  // singular values and their order
  for (int j = wave; j < N; j += JW) {
    const double* aj = A + (size_t)j * lda;
    double s2 = 0.0;
    for (int i = lane; i < M; i += 64) s2 = fma(aj[i], aj[i], s2);
    s2 = wave_sum(s2);
    if (lane == 0) sig[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < N; j += NT) {
    const double sj = sig[j];
    int rk = 0;
    for (int i = 0; i < N; ++i) rk += (sig[i] > sj) || (sig[i] == sj && i < j);
    rnk[j] = rk;
  }
  __syncthreads();
  for (int j = wave; j < N; j += JW) {
    const int rk = rnk[j];
    const double sj = sig[j];
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    const double* aj = A + (size_t)j * lda;
    double* uo = J.U + (size_t)rk * J.ldu;
    for (int i = lane; i < M; i += 64) uo[i] = aj[i] * inv;
    const double* vj = V + (size_t)j * N;
    for (int i = lane; i < N; i += 64) J.Vt[rk + (size_t)i * J.ldvt] = vj[i];
    if (lane == 0) J.S[rk] = sj;
  }
  if (tid == 0) J.info[0] = sweep < max_sweeps ? 0 : 1;
}
void jacobi_svd(const SvdJob* jobs, int njobs, int max_sweeps, bool in_lds, hipStream_t s) {
  if (njobs <= 0) return;
  if (in_lds)
    hipLaunchKernelGGL(jacobi_svd_kernel<true>, dim3(njobs), dim3(64 * JW), 0, s, jobs, max_sweeps);
  else
    hipLaunchKernelGGL(jacobi_svd_kernel<false>, dim3(njobs), dim3(64 * JW), 0, s, jobs, max_sweeps);
  HIPCHECK(hipGetLastError());
}

// Blocked one-sided Jacobi SVD: one tall matrix spread over many workgroups.  The N
// columns are cut into blocks of BJ = 8 (the last one narrower).  A sweep is one launch in
// which each workgroup rotates the pairs inside one block (the tournament of the
// one-workgroup kernel over the block's columns), then one launch per round of a
// round-robin tournament over the blocks, in which each workgroup takes two blocks and
// visits their cross pairs in BJ rounds: column k of the first block against column
// (k + t) mod BJ of the second in round t, so a round's pairs are disjoint and each
// of the BJ waves takes one.  Every column pair is thus visited once per sweep, with the
// pair test, rotation and zero-column rule of the one-workgroup kernel; the host ends a
// matrix's sweeps after one without a rotation.  A launch holds its blocks' columns of A
// and V in LDS, or in a cross launch the first block's in registers (one column per
// wave) and only the second block's in LDS.  A round's latency (the dot products, three wave sums and the rotation's
// square roots and divisions, one after another) bounds these kernels, not the issue
// rate: blocks of 8 columns (two waves per SIMD) measured faster than blocks of 16.
constexpr int kBJLds = 18432;  // doubles of LDS per workgroup (144 KiB)
constexpr int kBJ = 8;         // columns per block
bool jacobi_blocked_fits(int M, int N) {
  return N >= 2 && M >= N && N <= kJacobiMaxN && (long long)(M + N) * 2 * kBJ <= kBJLds;
}
// rotation of a column pair: cosine and sine from |a_p|^2, |a_q|^2 and a_p . a_q
__device__ __forceinline__ void bj_coeffs(double al, double be, double ga, double& c, double& sn) {
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  c = 1.0 / sqrt(1.0 + t * t);
  sn = c * t;
}
// one Jacobi rotation of the column pair (p, q) held in LDS, by one wave (wave-uniform
// arguments); returns whether it rotated.  With R > 0 (M, N <= 64 R) a lane loads its R
// rows of both columns at once; R = 0 walks the columns in a loop (same sums: a lane adds
// its rows in increasing order either way).
template <int R>
__device__ __forceinline__ bool bj_rotate(double* ap, double* aq, double* vp, double* vq, int M, int N, int lane,
                                          double tol, double zero2) {
  double al = 0.0, be = 0.0, ga = 0.0, c, sn;
  if constexpr (R > 0) {
    double x[R], y[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = lane + 64 * u;
      x[u] = i < M ? ap[i] : 0.0;
      y[u] = i < M ? aq[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      al = fma(x[u], x[u], al);
      be = fma(y[u], y[u], be);
      ga = fma(x[u], y[u], ga);
    }
    al = wave_sum(al);
    be = wave_sum(be);
    ga = wave_sum(ga);
    if (!(fabs(ga) > tol * sqrt(al * be)) || !(fmin(al, be) > zero2)) return false;
    bj_coeffs(al, be, ga, c, sn);
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = lane + 64 * u;
      if (i < M) {
        ap[i] = c * x[u] - sn * y[u];
        aq[i] = sn * x[u] + c * y[u];
      }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = lane + 64 * u;
      x[u] = i < N ? vp[i] : 0.0;
      y[u] = i < N ? vq[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = lane + 64 * u;
      if (i < N) {
        vp[i] = c * x[u] - sn * y[u];
        vq[i] = sn * x[u] + c * y[u];
      }
    }
  } else {
    for (int i = lane; i < M; i += 64) {
      const double x = ap[i], y = aq[i];
      al = fma(x, x, al);
      be = fma(y, y, be);
      ga = fma(x, y, ga);
    }
    al = wave_sum(al);
    be = wave_sum(be);
    ga = wave_sum(ga);
    if (!(fabs(ga) > tol * sqrt(al * be)) || !(fmin(al, be) > zero2)) return false;
    bj_coeffs(al, be, ga, c, sn);
    for (int i = lane; i < M; i += 64) {
      const double x = ap[i], y = aq[i];
      ap[i] = c * x - sn * y;
      aq[i] = sn * x + c * y;
    }
    for (int i = lane; i < N; i += 64) {
      const double x = vp[i], y = vq[i];
      vp[i] = c * x - sn * y;
      vq[i] = sn * x + c * y;
    }
  }
  return true;
}
// V = identity and |A|_F^2 of each matrix (one workgroup per matrix)
__global__ __launch_bounds__(64 * JW) void bj_init_kernel(const SvdJob* __restrict__ jobs, double* __restrict__ fro2) {
  const SvdJob J = jobs[blockIdx.x];
  const int M = J.M, N = J.N, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NT = 64 * JW;
  for (long long i = tid; i < (long long)N * N; i += NT) J.V[i] = (i % (N + 1) == 0) ? 1.0 : 0.0;
  __shared__ double fro_w[JW];
  double s2 = 0.0;
  for (int j = wave; j < N; j += JW)
    for (int i = lane; i < M; i += 64) s2 = fma(J.A[(size_t)j * J.lda + i], J.A[(size_t)j * J.lda + i], s2);
  s2 = wave_sum(s2);
  if (lane == 0) fro_w[wave] = s2;
  __syncthreads();
  if (tid == 0) {
    double f = 0.0;
    for (int w = 0; w < JW; ++w) f += fro_w[w];
    fro2[blockIdx.x] = f;
  }
}
// pairs inside block blockIdx.x of matrix act[blockIdx.y]
template <int BJ, int R>
__global__ __launch_bounds__(64 * BJ) void bj_within_kernel(const SvdJob* __restrict__ jobs,
                                                            const int* __restrict__ act,
                                                            const double* __restrict__ fro2, int* __restrict__ rot) {
  __shared__ double lds[kBJLds / 2];
  const int jb = act[blockIdx.y];
  const SvdJob J = jobs[jb];
  const int M = J.M, N = J.N, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NT = 64 * BJ;
  const int c0 = blockIdx.x * BJ;
  if (c0 >= N) return;
  const int w = min(BJ, N - c0);
  double* a = lds;                   // column k of the block at a + k M
  double* v = lds + (size_t)M * BJ;  // its column of V at v + k N
  for (int i = tid; i < M * w; i += NT) a[i] = J.A[(size_t)(c0 + i / M) * J.lda + i % M];
  for (int i = tid; i < N * w; i += NT) v[i] = J.V[(size_t)(c0 + i / N) * N + i % N];
  __syncthreads();
  const double tol = 2.2e-16 * (double)M, zero2 = tol * tol * fro2[jb];
  const int wp = w + (w & 1);
  bool any = false;
  for (int r = 0; r < wp - 1; ++r) {
    if (wave < wp / 2) {
      int p, q;
      if (wave == 0) { p = wp - 1; q = r; }
      else { p = (r + wave) % (wp - 1); q = (r - wave + wp - 1) % (wp - 1); }
      if (p < w && q < w)
        any |= bj_rotate<R>(a + (size_t)p * M, a + (size_t)q * M, v + (size_t)p * N, v + (size_t)q * N, M, N, lane,
                            tol, zero2);
    }
    __syncthreads();
  }
  for (int i = tid; i < M * w; i += NT) J.A[(size_t)(c0 + i / M) * J.lda + i % M] = a[i];
  for (int i = tid; i < N * w; i += NT) J.V[(size_t)(c0 + i / N) * N + i % N] = v[i];
  if (any && lane == 0) atomicAdd(rot + jb, 1);
}
// cross pairs of the two blocks that workgroup blockIdx.x meets in tournament round r.
// Wave k pairs column k of the first block with column (k + t) mod BJ of the second in
// round t.  With R > 0 (M, N <= 64 R) wave k keeps its column of the first block and of V
// in registers for the whole launch and only the second block is held in LDS; with R = 0
// both blocks are held in LDS.
template <int BJ, int R>
__global__ __launch_bounds__(64 * BJ) void bj_cross_kernel(const SvdJob* __restrict__ jobs,
                                                           const int* __restrict__ act,
                                                           const double* __restrict__ fro2, int* __restrict__ rot,
                                                           int r) {
  __shared__ double lds[R > 0 ? kBJLds / 2 : kBJLds];
  const int jb = act[blockIdx.y];
  const SvdJob J = jobs[jb];
  const int M = J.M, N = J.N, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NT = 64 * BJ;
  const int nb = (N + BJ - 1) / BJ, nbp = nb + (nb & 1);
  const int k = blockIdx.x;
  if (r >= nbp - 1 || k >= nbp / 2) return;
  int bi, bk;
  if (k == 0) { bi = nbp - 1; bk = r; }
  else { bi = (r + k) % (nbp - 1); bk = (r - k + nbp - 1) % (nbp - 1); }
  if (bi >= nb || bk >= nb) return;
  const int ci = bi * BJ, ck = bk * BJ, wi = min(BJ, N - ci), wk = min(BJ, N - ck);
  const double tol = 2.2e-16 * (double)M, zero2 = tol * tol * fro2[jb];
  bool any = false;
  if constexpr (R > 0) {
    // the second block's columns at a + j M and v + j N (j < wk)
    double* a = lds;
    double* v = lds + (size_t)M * BJ;
    for (int i = tid; i < M * wk; i += NT) a[i] = J.A[(size_t)(ck + i / M) * J.lda + i % M];
    for (int i = tid; i < N * wk; i += NT) v[i] = J.V[(size_t)(ck + i / N) * N + i % N];
    const int p = wave;
    const bool own = p < wi;
    double* gA = J.A + (size_t)(ci + (own ? p : 0)) * J.lda;
    double* gV = J.V + (size_t)(ci + (own ? p : 0)) * N;
    double x[R], vx[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = lane + 64 * u;
      x[u] = own && i < M ? gA[i] : 0.0;
      vx[u] = own && i < N ? gV[i] : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < BJ; ++t) {
      const int q = (p + t) % BJ;
      if (own && q < wk) {
        double* ay = a + (size_t)q * M;
        double* vy = v + (size_t)q * N;
        double y[R];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int u = 0; u < R; ++u) {
          const int i = lane + 64 * u;
          y[u] = i < M ? ay[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
          al = fma(x[u], x[u], al);
          be = fma(y[u], y[u], be);
          ga = fma(x[u], y[u], ga);
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (fabs(ga) > tol * sqrt(al * be) && fmin(al, be) > zero2) {
          double c, sn;
          bj_coeffs(al, be, ga, c, sn);
#pragma unroll
          for (int u = 0; u < R; ++u) {
            const int i = lane + 64 * u;
            const double xn = c * x[u] - sn * y[u], yn = sn * x[u] + c * y[u];
            x[u] = xn;
            if (i < M) ay[i] = yn;
          }
#pragma unroll
          for (int u = 0; u < R; ++u) {
            const int i = lane + 64 * u;
            y[u] = i < N ? vy[i] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < R; ++u) {
            const int i = lane + 64 * u;
            const double xn = c * vx[u] - sn * y[u], yn = sn * vx[u] + c * y[u];
            vx[u] = xn;
            if (i < N) vy[i] = yn;
          }
          any = true;
        }
      }
      __syncthreads();
    }
    if (own) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int i = lane + 64 * u;
        if (i < M) gA[i] = x[u];
        if (i < N) gV[i] = vx[u];
      }
    }
    for (int i = tid; i < M * wk; i += NT) J.A[(size_t)(ck + i / M) * J.lda + i % M] = a[i];
    for (int i = tid; i < N * wk; i += NT) J.V[(size_t)(ck + i / N) * N + i % N] = v[i];
  } else {
    // columns of the first block at a + j M (j < wi), of the second at a + (BJ + j) M; V alike
    double* a = lds;
    double* v = lds + (size_t)M * 2 * BJ;
    for (int i = tid; i < M * wi; i += NT) a[i] = J.A[(size_t)(ci + i / M) * J.lda + i % M];
    for (int i = tid; i < M * wk; i += NT) a[(size_t)M * BJ + i] = J.A[(size_t)(ck + i / M) * J.lda + i % M];
    for (int i = tid; i < N * wi; i += NT) v[i] = J.V[(size_t)(ci + i / N) * N + i % N];
    for (int i = tid; i < N * wk; i += NT) v[(size_t)N * BJ + i] = J.V[(size_t)(ck + i / N) * N + i % N];
    __syncthreads();
    for (int t = 0; t < BJ; ++t) {
      const int p = wave, q = (wave + t) % BJ;
      if (p < wi && q < wk)
        any |= bj_rotate<0>(a + (size_t)p * M, a + (size_t)(BJ + q) * M, v + (size_t)p * N,
                            v + (size_t)(BJ + q) * N, M, N, lane, tol, zero2);
      __syncthreads();
    }
    for (int i = tid; i < M * wi; i += NT) J.A[(size_t)(ci + i / M) * J.lda + i % M] = a[i];
    for (int i = tid; i < M * wk; i += NT) J.A[(size_t)(ck + i / M) * J.lda + i % M] = a[(size_t)M * BJ + i];
    for (int i = tid; i < N * wi; i += NT) J.V[(size_t)(ci + i / N) * N + i % N] = v[i];
    for (int i = tid; i < N * wk; i += NT) J.V[(size_t)(ck + i / N) * N + i % N] = v[(size_t)N * BJ + i];
  }
  if (any && lane == 0) atomicAdd(rot + jb, 1);
}
// one sweep: the pairs inside every block, then the tournament rounds over the blocks
template <int BJ, int R>
void bj_sweep(const SvdJob* jobs, const int* act, const double* fro2, int* rot, int nbmax, int nact, hipStream_t s) {
  const int nbpmax = nbmax + (nbmax & 1);
  hipLaunchKernelGGL((bj_within_kernel<BJ, R>), dim3(nbmax, nact), dim3(64 * BJ), 0, s, jobs, act, fro2, rot);
  HIPCHECK(hipGetLastError());
  for (int r = 0; r < nbpmax - 1; ++r) {
    hipLaunchKernelGGL((bj_cross_kernel<BJ, R>), dim3(nbpmax / 2, nact), dim3(64 * BJ), 0, s, jobs, act, fro2, rot,
                       r);
    HIPCHECK(hipGetLastError());
  }
}
// singular triplets in decreasing order of sigma (ties by column index), as the
// one-workgroup kernel writes them; info = 1 for a matrix still rotating in its last sweep
__global__ __launch_bounds__(64 * JW) void bj_finish_kernel(const SvdJob* __restrict__ jobs,
                                                            const int* __restrict__ rot) {
  __shared__ double sig[kJacobiMaxN];
  __shared__ int rnk[kJacobiMaxN];
  const SvdJob J = jobs[blockIdx.x];
  const int M = J.M, N = J.N, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NT = 64 * JW;
  for (int j = wave; j < N; j += JW) {
    const double* aj = J.A + (size_t)j * J.lda;
    double s2 = 0.0;
    for (int i = lane; i < M; i += 64) s2 = fma(aj[i], aj[i], s2);
    s2 = wave_sum(s2);
    if (lane == 0) sig[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < N; j += NT) {
    const double sj = sig[j];
    int rk = 0;
    for (int i = 0; i < N; ++i) rk += (sig[i] > sj) || (sig[i] == sj && i < j);
    rnk[j] = rk;
  }
  __syncthreads();
  for (int j = wave; j < N; j += JW) {
    const int rk = rnk[j];
    const double sj = sig[j];
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    const double* aj = J.A + (size_t)j * J.lda;
    double* uo = J.U + (size_t)rk * J.ldu;
    for (int i = lane; i < M; i += 64) uo[i] = aj[i] * inv;
    const double* vj = J.V + (size_t)j * N;
    for (int i = lane; i < N; i += 64) J.Vt[rk + (size_t)i * J.ldvt] = vj[i];
    if (lane == 0) J.S[rk] = sj;
  }
  if (tid == 0) J.info[0] = rot[blockIdx.x] > 0 ? 1 : 0;
}
void jacobi_svd_blocked(const SvdJob* jobs, const SvdJob* jobs_host, int njobs, int rows, int max_sweeps,
                        double* fro2, int* rot, int* act_dev, hipStream_t s) {
  if (njobs <= 0) return;
  int nbmax = 1, mmax = 1;
  for (int j = 0; j < njobs; ++j) {
    const SvdJob& J = jobs_host[j];
    if (!jacobi_blocked_fits(J.M, J.N) || J.V == nullptr || J.lda < J.M || J.ldu < J.M || J.ldvt < J.N)
      throw std::logic_error("jacobi_svd_blocked: a matrix shape the blocked kernels do not take");
    nbmax = std::max(nbmax, (J.N + kBJ - 1) / kBJ);
    mmax = std::max(mmax, J.M);
  }
  // rows per lane held in registers by the pair kernels: 4 or 9, or 0 (loops over LDS)
  const int R = rows >= 0 ? rows : mmax <= 256 ? 4 : mmax <= 576 ? 9 : 0;
  if ((R != 0 && R != 4 && R != 9) || (R != 0 && mmax > 64 * R))
    throw std::logic_error("jacobi_svd_blocked: rows per lane must be 0, 4 or 9 and cover every matrix");
  hipLaunchKernelGGL(bj_init_kernel, dim3(njobs), dim3(64 * JW), 0, s, jobs, fro2);
  HIPCHECK(hipGetLastError());
  fill(rot, sizeof(int) * njobs, s);  // read by the finish kernel even if no sweep runs
  std::vector<int> act(njobs), rh(njobs);
  for (int j = 0; j < njobs; ++j) act[j] = j;
  for (int sweep = 0; sweep < max_sweeps && !act.empty(); ++sweep) {
    const int nact = (int)act.size();
    HIPCHECK(hipMemcpyAsync(act_dev, act.data(), sizeof(int) * nact, hipMemcpyHostToDevice, s));
    fill(rot, sizeof(int) * njobs, s);
    if (R == 4) bj_sweep<kBJ, 4>(jobs, act_dev, fro2, rot, nbmax, nact, s);
    else if (R == 9) bj_sweep<kBJ, 9>(jobs, act_dev, fro2, rot, nbmax, nact, s);
    else bj_sweep<kBJ, 0>(jobs, act_dev, fro2, rot, nbmax, nact, s);
    HIPCHECK(hipMemcpyAsync(rh.data(), rot, sizeof(int) * njobs, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    std::vector<int> next;
    for (int j : act)
      if (rh[j] > 0) next.push_back(j);
    act.swap(next);
  }
  hipLaunchKernelGGL(bj_finish_kernel, dim3(njobs), dim3(64 * JW), 0, s, jobs, rot);
  HIPCHECK(hipGetLastError());
}

// out = sum_i c[i] V_i; with VEC = 2 a thread produces two adjacent entries from 16-byte
// loads, and the vectors are taken four at a time so that four loads are in flight
template <int VEC>
__global__ __launch_bounds__(256) void lincomb_kernel(const double* __restrict__ V, size_t ldv, int m,
                                                      const double* __restrict__ c, double* __restrict__ out,
                                                      size_t n) {
  const size_t nv = n / VEC;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < nv; k += (size_t)gridDim.x * blockDim.x) {
    if constexpr (VEC == 2) {
      double2 s = {0.0, 0.0};
      int i = 0;
      for (; i + 4 <= m; i += 4) {
        double2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = reinterpret_cast<const double2*>(V + (size_t)(i + u) * ldv)[k];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          s.x = fma(c[i + u], v[u].x, s.x);
          s.y = fma(c[i + u], v[u].y, s.y);
        }
      }
      for (; i < m; ++i) {
        const double2 v = reinterpret_cast<const double2*>(V + (size_t)i * ldv)[k];
        s.x = fma(c[i], v.x, s.x);
        s.y = fma(c[i], v.y, s.y);
      }
      reinterpret_cast<double2*>(out)[k] = s;
    } else {
      double s = 0.0;
      for (int i = 0; i < m; ++i) s = fma(c[i], V[(size_t)i * ldv + k], s);
      out[k] = s;
    }
  }
}
void lincomb(const double* V, size_t ldv, int m, const double* c_dev, double* out, size_t n, hipStream_t s) {
  if (!n) return;
  const bool vec2 = n % 2 == 0 && ldv % 2 == 0 && (uintptr_t)V % 16 == 0 && (uintptr_t)out % 16 == 0;
  if (vec2)
    hipLaunchKernelGGL(lincomb_kernel<2>, dim3(nblocks(n / 2)), dim3(256), 0, s, V, ldv, m, c_dev, out, n);
  else
    hipLaunchKernelGGL(lincomb_kernel<1>, dim3(nblocks(n)), dim3(256), 0, s, V, ldv, m, c_dev, out, n);
  HIPCHECK(hipGetLastError());
}

__global__ void cvt_d2f(const double* a, float* b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}
__global__ void cvt_f2d(const float* a, double* b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (double)a[i];
}
__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__global__ void cvt_d2bf(const double* a, uint16_t* b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = f32_to_bf16_rne((float)a[i]);
}
void convert_f64_f32(const double* a, float* b, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(cvt_d2f, dim3(nblocks(n)), dim3(256), 0, s, a, b, n);
  HIPCHECK(hipGetLastError());
}
void convert_f64_f32_op(const double* a, float* b, size_t n, hipStream_t s) { convert_f64_f32(a, b, n, s); }
void convert_f32_f64(const float* a, double* b, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(cvt_f2d, dim3(nblocks(n)), dim3(256), 0, s, a, b, n);
  HIPCHECK(hipGetLastError());
}
void convert_f64_bf16(const double* a, uint16_t* b, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(cvt_d2bf, dim3(nblocks(n)), dim3(256), 0, s, a, b, n);
  HIPCHECK(hipGetLastError());
}
__global__ void cvt_d2bff(const double* a, float* b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = __uint_as_float((uint32_t)f32_to_bf16_rne((float)a[i]) << 16);
}
void convert_f64_bf16f32(const double* a, float* b, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(cvt_d2bff, dim3(nblocks(n)), dim3(256), 0, s, a, b, n);
  HIPCHECK(hipGetLastError());
}

__global__ void gather_blocks_kernel(const double* __restrict__ M, long long ldm, const int* __restrict__ rows,
                                     const int* __restrict__ cols, const GatherBlk* __restrict__ blks,
                                     double* __restrict__ dst) {
  const GatherBlk b = blks[blockIdx.x];
  for (int e = threadIdx.x; e < b.m * b.n; e += blockDim.x) {
    const int j = e / b.m, i = e - j * b.m;
    const long long d = b.trans ? b.dst + (long long)i * b.ld + j : b.dst + (long long)j * b.ld + i;
    dst[d] = M[(long long)rows[b.roff + i] * ldm + cols[b.coff + j]];
  }
}
void gather_blocks(const double* M, long long ldm, const int* rows, const int* cols, const GatherBlk* blks, int nblk,
                   double* dst, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(gather_blocks_kernel, dim3(nblk), dim3(256), 0, s, M, ldm, rows, cols, blks, dst);
  HIPCHECK(hipGetLastError());
}
__global__ void scatter_left_kernel(const ScatterBlk* __restrict__ blks, const int* __restrict__ rows,
                                    double* __restrict__ left, long long ldl, int mode) {
  const ScatterBlk b = blks[blockIdx.x];
  for (int e = threadIdx.x; e < b.m * b.t; e += blockDim.x) {
    const int j = e / b.m, i = e - j * b.m;
    double v = b.U[i * b.us_i + j * b.us_j];
    if (mode == 1) v *= b.S[j];
    left[(long long)rows[b.roff + i] * ldl + b.off + j] = v;
  }
}
__global__ void scatter_right_kernel(const ScatterBlk* __restrict__ blks, const int* __restrict__ cols,
                                     double* __restrict__ right, long long ldr, int mode) {
  const ScatterBlk b = blks[blockIdx.x];
  for (int e = threadIdx.x; e < b.t * b.n; e += blockDim.x) {
    const int c = e / b.t, j = e - c * b.t;
    double v = b.Vt[j * b.vs_j + c * b.vs_c];
    if (mode == 0) v *= b.S[j];
    right[(long long)(b.off + j) * ldr + cols[b.coff + c]] = v;
  }
}
void scatter_factors(const ScatterBlk* blks, int nblk, const int* rows, const int* cols, double* left, long long ldl,
                     double* right, long long ldr, int mode, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(scatter_left_kernel, dim3(nblk), dim3(256), 0, s, blks, rows, left, ldl, mode);
  HIPCHECK(hipGetLastError());
  hipLaunchKernelGGL(scatter_right_kernel, dim3(nblk), dim3(256), 0, s, blks, cols, right, ldr, mode);
  HIPCHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Householder LQ of sector blocks (one workgroup of HHW waves per block): the
// unblocked algorithm, each reflector from one row, the trailing rows updated
// one wave per row; then Q formed by applying the reflectors in reverse order
// to the first k rows of the identity.  The block lives in global memory (L2),
// the current reflector in LDS.  A row's update waits on its loads from L2, so the
// rows a workgroup updates at once set the pace: 16 waves rather than 4.
// ---------------------------------------------------------------------------
__device__ inline double hh_wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
constexpr int HHW = 16;       // waves per workgroup
constexpr int HHT = 64 * HHW;  // threads per workgroup
__device__ inline double hh_block_sum(double x, double* red) {
  x = hh_wave_sum(x);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < HHW; ++w) t += red[w];
  __syncthreads();
  return t;
}
__global__ __launch_bounds__(HHT) void householder_lq_kernel(const double* __restrict__ W, long long sWr, long long sWc,
                                                             const int* __restrict__ rows, const int* __restrict__ cols,
                                                             const int* __restrict__ nmap, const HhBlk* __restrict__ blks,
                                                             double* __restrict__ ws,
                                                             double* __restrict__ Lout, long long sLr, long long sLc,
                                                             double* __restrict__ Qout, long long sQr, long long sQc) {
  __shared__ double v[HH_MAXN];
  __shared__ double red[HHW];
  const HhBlk b = blks[blockIdx.x];
  const int m = b.m, n = b.n, k = m < n ? m : n;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* A = ws + b.ws;
  double* X = A + (long long)m * n;
  double* tau = X + (long long)k * n;
  const int* rw = rows + b.roff;
  const int* cl = cols + b.coff;
  const int* nw = nmap + b.noff;
  for (long long e = tid; e < (long long)m * n; e += HHT) {
    const int r = (int)(e / n), c = (int)(e - (long long)r * n);
    A[e] = W[(long long)rw[r] * sWr + (long long)cl[c] * sWc];
  }
  __syncthreads();
  // factorisation
  for (int i = 0; i < k; ++i) {
    double* Ai = A + (long long)i * n;
    double part = 0.0;
    for (int c = i + 1 + tid; c < n; c += HHT) part += Ai[c] * Ai[c];
    const double sig = hh_block_sum(part, red);
    const double alpha = Ai[i];
    double t = 0.0, beta = alpha, scl = 0.0;
    if (sig > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + sig), alpha);
      t = (beta - alpha) / beta;
      scl = 1.0 / (alpha - beta);
    }
    for (int c = i + tid; c < n; c += HHT) v[c - i] = c == i ? 1.0 : Ai[c] * scl;
    __syncthreads();
    if (t != 0.0) {
      for (int r = i + 1 + wv; r < m; r += HHW) {
        double* Ar = A + (long long)r * n;
        double d = 0.0;
        for (int c = i + lane; c < n; c += 64) d += Ar[c] * v[c - i];
        d = hh_wave_sum(d) * t;
        for (int c = i + lane; c < n; c += 64) Ar[c] -= d * v[c - i];
      }
    }
    for (int c = i + 1 + tid; c < n; c += HHT) Ai[c] = v[c - i];
    if (tid == 0) {
      Ai[i] = beta;
      tau[i] = t;
    }
    __syncthreads();
  }
  // Q = [I_k 0] H(k-1) ... H(0): when H(i) is applied only rows >= i and columns >= i change
  for (long long e = tid; e < (long long)k * n; e += HHT) {
    const int r = (int)(e / n), c = (int)(e - (long long)r * n);
    X[e] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const double t = tau[i];
    if (t == 0.0) continue;
    const double* Ai = A + (long long)i * n;
    for (int c = i + tid; c < n; c += HHT) v[c - i] = c == i ? 1.0 : Ai[c];
    __syncthreads();
    for (int r = i + wv; r < k; r += HHW) {
      double* Xr = X + (long long)r * n;
      double d = 0.0;
      for (int c = i + lane; c < n; c += 64) d += Xr[c] * v[c - i];
      d = hh_wave_sum(d) * t;
      for (int c = i + lane; c < n; c += 64) Xr[c] -= d * v[c - i];
    }
    __syncthreads();
  }
  for (long long e = tid; e < (long long)m * k; e += HHT) {
    const int r = (int)(e / k), c = (int)(e - (long long)r * k);
    if (c <= r) Lout[(long long)rw[r] * sLr + (long long)nw[c] * sLc] = A[(long long)r * n + c];
  }
  for (long long e = tid; e < (long long)k * n; e += HHT) {
    const int r = (int)(e / n), c = (int)(e - (long long)r * n);
    Qout[(long long)nw[r] * sQr + (long long)cl[c] * sQc] = X[e];
  }
}
void householder_lq(const double* W, long long sWr, long long sWc, const int* rows, const int* cols, const int* nmap,
                    const HhBlk* blks, int nblk, double* ws, double* Lout, long long sLr, long long sLc, double* Qout,
                    long long sQr, long long sQc, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(householder_lq_kernel, dim3(nblk), dim3(HHT), 0, s, W, sWr, sWc, rows, cols, nmap, blks, ws, Lout,
                     sLr, sLc, Qout, sQr, sQc);
  HIPCHECK(hipGetLastError());
}

__global__ void gather2d_kernel(const double* src, long long lds, const int* rows, int nr, const int* cols, int nc,
                                double* dst, bool colmajor) {
  const long long tot = (long long)nr * nc;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot; t += (long long)gridDim.x * blockDim.x) {
    int i, j;
    if (colmajor) { i = (int)(t % nr); j = (int)(t / nr); }
    else { i = (int)(t / nc); j = (int)(t % nc); }
    const double v = src[(long long)rows[i] * lds + cols[j]];
    if (colmajor) dst[(long long)j * nr + i] = v; else dst[(long long)i * nc + j] = v;
  }
}
void gather2d(const double* src, long long lds, const int* rows, int nr, const int* cols, int nc, double* dst,
              bool colmajor, hipStream_t s) {
  if (nr <= 0 || nc <= 0) return;
  hipLaunchKernelGGL(gather2d_kernel, dim3(nblocks((size_t)nr * nc)), dim3(256), 0, s, src, lds, rows, nr, cols, nc,
                     dst, colmajor);
  HIPCHECK(hipGetLastError());
}

__global__ void scatter2d_kernel(const double* src, long long sr, long long sc, const int* rows, int nr,
                                 const int* cols, int nc, double* dst, long long ldd, double alpha, const double* rs,
                                 const double* cs, int tri) {
  const long long tot = (long long)nr * nc;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot; t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t % nr);
    const int j = (int)(t / nr);
    double v = 0.0;
    if (tri == 0 || (tri == 1 && i <= j) || (tri == 2 && j <= i)) {
      v = alpha * src[i * sr + j * sc];
      if (rs) v *= rs[i];
      if (cs) v *= cs[j];
    }
    dst[(long long)rows[i] * ldd + cols[j]] = v;
  }
}
void scatter2d(const double* src, long long sr, long long sc, const int* rows, int nr, const int* cols, int nc,
               double* dst, long long ldd, double alpha, const double* rs, const double* cs, int tri, hipStream_t s) {
  if (nr <= 0 || nc <= 0) return;
  hipLaunchKernelGGL(scatter2d_kernel, dim3(nblocks((size_t)nr * nc)), dim3(256), 0, s, src, sr, sc, rows, nr, cols,
                     nc, dst, ldd, alpha, rs, cs, tri);
  HIPCHECK(hipGetLastError());
}

__global__ void permute_core_kernel(const double* in, int irp, const int* pl, const int* pr, int rl, int rr,
                                    double* out, int orp) {
  const long long tot = (long long)rl * 4 * rr;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot; t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t % rr);
    const long long r = t / rr;
    const int s = (int)(r % 4);
    const int a = (int)(r / 4);
    out[((long long)a * 4 + s) * orp + b] = in[((long long)pl[a] * 4 + s) * irp + pr[b]];
  }
}
void permute_core(const double* in, int irp, const int* pl, const int* pr, int rl, int rr, double* out, int orp,
                  hipStream_t s) {
  if ((long long)rl * rr == 0) return;
  hipLaunchKernelGGL(permute_core_kernel, dim3(nblocks((size_t)rl * 4 * rr)), dim3(256), 0, s, in, irp, pl, pr, rl, rr,
                     out, orp);
  HIPCHECK(hipGetLastError());
}

__global__ void copy3d_kernel(const double* src, long long s0, long long s1, double* dst, long long d0, long long d1,
                              int n0, int n1, int n2, double alpha, int acc) {
  const long long tot = (long long)n0 * n1 * n2;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot; t += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(t % n2);
    const long long r = t / n2;
    const int j = (int)(r % n1);
    const int i = (int)(r / n1);
    const double v = alpha * src[i * s0 + j * s1 + k];
    double* d = dst + (i * d0 + j * d1 + k);
    *d = acc ? *d + v : v;
  }
}
void copy3d(const double* src, long long s0, long long s1, double* dst, long long d0, long long d1, int n0, int n1,
            int n2, double alpha, hipStream_t s, bool accumulate) {
  if (n0 <= 0 || n1 <= 0 || n2 <= 0) return;
  hipLaunchKernelGGL(copy3d_kernel, dim3(nblocks((size_t)n0 * n1 * n2)), dim3(256), 0, s, src, s0, s1, dst, d0, d1, n0,
                     n1, n2, alpha, accumulate ? 1 : 0);
  HIPCHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// gradient of the sparse MPO entries (backward of the mixing stages)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void entry_grad_kernel(const int* gch, const int* tch, const T* G, long long g_cs,
                                                         const T* Tin, long long t_cs, int O, int I, double* gop) {
  const int e = blockIdx.x;
  const T* g = G + (long long)gch[e] * g_cs;
  const T* t = Tin + (long long)tch[e] * t_cs;
  const long long npos = (long long)O * I;
  double acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0;
  for (long long p = threadIdx.x; p < npos; p += blockDim.x) {
    const long long o = p / I, i = p % I;
    const long long off = o * 4LL * I + i;
    double gv[4], tv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      gv[s] = (double)g[off + s * (long long)I];
      tv[s] = (double)t[off + s * (long long)I];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a * 4 + b] += gv[a] * tv[b];
  }
  __shared__ double red[256];
  for (int j = 0; j < 16; ++j) {
    red[threadIdx.x] = acc[j];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) gop[16LL * e + j] += red[0];
    __syncthreads();
  }
}

template <typename T>
void entry_grad(int nnz, const int* gch, const int* tch, const T* G, long long g_cs, const T* Tin, long long t_cs,
                int O, int I, double* gop, hipStream_t s) {
  if (nnz <= 0) return;
  if (!gch || !tch || !G || !Tin || !gop) throw std::runtime_error("entry_grad: null operand");
  hipLaunchKernelGGL((entry_grad_kernel<T>), dim3(nnz), dim3(256), 0, s, gch, tch, G, g_cs, Tin, t_cs, O, I, gop);
  HIPCHECK(hipGetLastError());
}
template void entry_grad<double>(int, const int*, const int*, const double*, long long, const double*, long long, int,
                                 int, double*, hipStream_t);

__global__ void transpose_kernel(const double* in, double* out, int n, int r, int c) {
  const long long tot = (long long)n * r * c;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot; t += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(t % c);
    const long long q = t / c;
    const int i = (int)(q % r);
    const long long b = q / r;
    out[(b * c + j) * r + i] = in[t];
  }
}
void transpose_batched(const double* in, double* out, int n, int r, int c, hipStream_t s) {
  if ((long long)n * r * c == 0) return;
  hipLaunchKernelGGL(transpose_kernel, dim3(nblocks((size_t)n * r * c)), dim3(256), 0, s, in, out, n, r, c);
  HIPCHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// diagonal of the effective Hamiltonian (Davidson preconditioner)
// ---------------------------------------------------------------------------
__global__ void diag_extract_kernel(const double* E, int R, int r, double* out) {
  const long long tot = (long long)R * r;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot; t += (long long)gridDim.x * blockDim.x) {
    const long long c = t / r, a = t % r;
    out[t] = E[(c * r + a) * r + a];
  }
}
void diag_extract(const double* E, int R, int r, double* out, hipStream_t s) {
  if ((long long)R * r == 0) return;
  hipLaunchKernelGGL(diag_extract_kernel, dim3(nblocks((size_t)R * r)), dim3(256), 0, s, E, R, r, out);
  HIPCHECK(hipGetLastError());
}

// out[c][n][s] (state_inner) or out[c][s][n]: sum over entries of op[e][s][s] * in[src[e]][n]
__global__ void diag_mix_kernel(int nout, const int* ptr, const int* src, const double* op, const double* in, int n,
                                double* out, bool state_inner) {
  const long long tot = (long long)nout * n;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot; t += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(t / n), a = (int)(t % n);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int e = ptr[c]; e < ptr[c + 1]; ++e) {
      const double v = in[(long long)src[e] * n + a];
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] += op[16LL * e + 5 * s] * v;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (state_inner) out[((long long)c * n + a) * 4 + s] = acc[s];
      else out[((long long)c * 4 + s) * n + a] = acc[s];
    }
  }
}
void diag_mix(int nout, const int* ptr, const int* src, const double* op, const double* in, int n, double* out,
              bool state_inner, hipStream_t s) {
  if ((long long)nout * n == 0) return;
  hipLaunchKernelGGL(diag_mix_kernel, dim3(nblocks((size_t)nout * n)), dim3(256), 0, s, nout, ptr, src, op, in, n, out,
                     state_inner);
  HIPCHECK(hipGetLastError());
}

// t = mask ? r / (theta - d) : 0, with |theta - d| clamped from below
__global__ void precond_kernel(double* t, const double* r, const double* d, double theta, const uint8_t* m, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double den = theta - d[i];
    if (fabs(den) < 1e-3) den = den < 0 ? -1e-3 : 1e-3;
    t[i] = (!m || m[i]) ? r[i] / den : 0.0;
  }
}
void precond(double* t, const double* r, const double* d, double theta, const uint8_t* m, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(precond_kernel, dim3(nblocks(n)), dim3(256), 0, s, t, r, d, theta, m, n);
  HIPCHECK(hipGetLastError());
}

}  // namespace tt
