// Quantum-number block-sparse two-site effective-Hamiltonian product:
// per-window plan (host) and the four device stages.  The layout is described
// in bsheff.h.
#include "bsheff.h"

#include <atomic>

#include <algorithm>
#include <cstdio>
#include <map>
#include <numeric>
#include <stdexcept>

namespace tt {

#define BSCHECK(x)                                                                   \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) throw tt::HipError(std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

namespace {

const Q2 kSiteQ[4] = {{0, 0}, {1, 1}, {1, -1}, {2, 0}};  // |0>, |up>, |dn>, |up dn>: (N, 2Sz)
inline Q2 add(Q2 a, Q2 b) { return {a[0] + b[0], a[1] + b[1]}; }
inline Q2 sub(Q2 a, Q2 b) { return {a[0] - b[0], a[1] - b[1]}; }

constexpr int TILE = 64;       // output tile edge of the stage-1 and stage-4 kernels
constexpr int LW_ROWS = 128;   // rows per workgroup of the left-operator GEMM
constexpr int KT = 32;         // K slice staged in LDS
constexpr int MIX_COLS = 256;  // spectator columns per mix workgroup (one per thread)
constexpr int MIX_ROWS = 64;   // output rows per mix workgroup
constexpr int KSPLIT = 2048;   // K chunk of one stage-4 workgroup
constexpr int HEAVY_MIN = 32;  // output rows with more operator entries go through the dense GEMM
constexpr int MIX_STAGE = 32;  // input rows a mix workgroup stages in LDS (>= HEAVY_MIN: any light row fits)

struct Sectors {
  std::vector<Q2> q;
  std::vector<int> off, n;
  std::map<Q2, int> id;
  int find(Q2 c) const {
    auto it = id.find(c);
    return it == id.end() ? -1 : it->second;
  }
};

// sectors of a label list; false if equal charges are not contiguous
bool make_sectors(const Labels& lab, Sectors& s) {
  for (int i = 0; i < (int)lab.size(); ++i) {
    if (i == 0 || lab[i] != lab[i - 1]) {
      if (s.id.count(lab[i])) return false;
      s.id[lab[i]] = (int)s.q.size();
      s.q.push_back(lab[i]);
      s.off.push_back(i);
      s.n.push_back(0);
    }
    s.n.back()++;
  }
  return true;
}

// sector index of a charge by table lookup (-1: none); the plan tables query it millions of times
struct QLook {
  int lo0 = 0, lo1 = 0, w0 = 0, w1 = 0;
  std::vector<int> t;
  explicit QLook(const Sectors& S) {
    if (S.q.empty()) return;
    int hi0 = S.q[0][0], hi1 = S.q[0][1];
    lo0 = hi0;
    lo1 = hi1;
    for (const Q2& q : S.q) {
      lo0 = std::min(lo0, q[0]); hi0 = std::max(hi0, q[0]);
      lo1 = std::min(lo1, q[1]); hi1 = std::max(hi1, q[1]);
    }
    w0 = hi0 - lo0 + 1;
    w1 = hi1 - lo1 + 1;
    t.assign((size_t)w0 * w1, -1);
    for (int i = 0; i < (int)S.q.size(); ++i) t[(size_t)(S.q[i][0] - lo0) * w1 + (S.q[i][1] - lo1)] = i;
  }
  int operator()(Q2 q) const {
    const int a = q[0] - lo0, b = q[1] - lo1;
    return (a < 0 || b < 0 || a >= w0 || b >= w1) ? -1 : t[(size_t)a * w1 + b];
  }
};

template <class V>
void up(DevMem& d, const std::vector<V>& v, hipStream_t s) {
  upload(d, v.data(), v.size() * sizeof(V), s);
}

__device__ inline float bf16_round(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// element loads and stores of the two precontracted-operator GEMMs: FP64, FP32, or
// bfloat16 storage (uint16_t bit patterns, FP32 arithmetic, round to nearest even)
__device__ inline double ldv(const double* p, long long i) { return p[i]; }
__device__ inline float ldv(const float* p, long long i) { return p[i]; }
__device__ inline float ldv(const uint16_t* p, long long i) { return __uint_as_float((uint32_t)p[i] << 16); }
__device__ inline void stv(double* p, long long i, double v) { p[i] = v; }
__device__ inline void stv(float* p, long long i, float v) { p[i] = v; }
__device__ inline void stv(uint16_t* p, long long i, float v) { p[i] = (uint16_t)(__float_as_uint(bf16_round(v)) >> 16); }
// a run of N consecutive elements from a 16-byte aligned address, as vector loads
template <int N>
__device__ inline void ldrun(const float* p, float (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N / 4; ++i) {
    const float4 q = reinterpret_cast<const float4*>(p)[i];
    v[4 * i] = q.x; v[4 * i + 1] = q.y; v[4 * i + 2] = q.z; v[4 * i + 3] = q.w;
  }
}
template <int N>
__device__ inline void ldrun(const double* p, double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const double2 q = reinterpret_cast<const double2*>(p)[i];
    v[2 * i] = q.x; v[2 * i + 1] = q.y;
  }
}
template <int N>
__device__ inline void ldrun(const uint16_t* p, float (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N / 8; ++i) {
    const uint4 q = reinterpret_cast<const uint4*>(p)[i];
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      v[8 * i + 2 * h] = __uint_as_float(w[h] << 16);
      v[8 * i + 2 * h + 1] = __uint_as_float(w[h] & 0xffff0000u);
    }
  }
}

// ---------------------------------------------------------------------------
// stage 1: T1[(A, s1)][spec(a', s2, b) + i' n_b + j] = sum_a L_A[a'][a] x[a][s1][s2][b]
// for each left sector alpha (rows (A, i') with a' in alpha + d_A, columns
// (s1, s2, j) with b in alpha + q(s1) + q(s2)).
// ---------------------------------------------------------------------------
// One stage-1 tile on the matrix cores.  The row and column descriptors
// of the tile are read once into LDS, the 64 x 64 product is formed with
// 16 x 16 x 4 MFMA blocks (K is one ket sector, a few slices at most) and
// staged in LDS, then written with consecutive threads on consecutive columns.
template <typename T>
__device__ inline void s1_mfma(T a, T b, T (&c)[4]);
template <>
__device__ inline void s1_mfma<float>(float a, float b, float (&c)[4]) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  v4 x = {c[0], c[1], c[2], c[3]};
  x = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, x, 0, 0, 0);
  c[0] = x[0]; c[1] = x[1]; c[2] = x[2]; c[3] = x[3];
}
template <>
__device__ inline void s1_mfma<double>(double a, double b, double (&c)[4]) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  v4 x = {c[0], c[1], c[2], c[3]};
  x = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, x, 0, 0, 0);
  c[0] = x[0]; c[1] = x[1]; c[2] = x[2]; c[3] = x[3];
}

template <typename T>
__global__ __launch_bounds__(256) void stage1_mfma_kernel(
    const int4* __restrict__ tiles, const BsAlpha* __restrict__ al, const long long* __restrict__ rsrc,
    const int4* __restrict__ rinfo, const int4* __restrict__ cinfo, const long long* __restrict__ rowpart,
    const long long* __restrict__ specoff, const int* __restrict__ nbeta, int nbe, const T* __restrict__ L, long long nL,
    const T* __restrict__ x, long long nx, long long xld, T* __restrict__ out, long long nout, int* __restrict__ err) {
  constexpr int KS = sizeof(T) == 4 ? 32 : 16;
  constexpr int RUNL = KS / 4;
  const int4 t = tiles[blockIdx.x];
  const BsAlpha a = al[t.x];
  const int m0 = t.y, c0 = t.z;
  __shared__ T As[KS][TILE + 4];
  __shared__ T Bs[KS][TILE + 4];
  __shared__ T Cs[TILE][TILE + 1];
  __shared__ long long rs[TILE];
  __shared__ int4 ri[TILE], ci[TILE];
  __shared__ int nb[TILE];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int mrows = min(TILE, a.M - m0), ncols = min(TILE, a.N - c0);
  if (tid < TILE) {
    if (tid < mrows) {
      rs[tid] = rsrc[a.row0 + m0 + tid];
      ri[tid] = rinfo[a.row0 + m0 + tid];  // {A, i', alpha', -}
    }
  } else if (tid < 2 * TILE) {
    const int c = tid - TILE;
    if (c < ncols) {
      const int4 q = cinfo[a.col0 + c0 + c];  // {x column, s1*4+s2, beta, j}
      ci[c] = q;
      nb[c] = nbeta[q.z];
    }
  }
  __syncthreads();
  const int nblk = (ncols + 15) >> 4;
  const int ar = tid >> 2, ak = (tid & 3) * RUNL;
  const int bk = tid / (TILE / RUNL), bn = (tid % (TILE / RUNL)) * RUNL;
  T acc[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[j][v] = T(0);
  for (int k0 = 0; k0 < a.K; k0 += KS) {
#pragma unroll
    for (int u = 0; u < RUNL; ++u) {
      const int k = k0 + ak + u;
      T v = T(0);
      if (ar < mrows && k < a.K) {
        const long long q = rs[ar] + k;
        if (q >= 0 && q < nL) v = L[q]; else err[0] = 1;
      }
      As[ak + u][ar] = v;
    }
    const int kb = k0 + bk;
#pragma unroll
    for (int u = 0; u < RUNL; ++u) {
      const int c = bn + u;
      T v = T(0);
      if (c < ncols && kb < a.K) {
        const long long q = (long long)(a.oal + kb) * xld + ci[c].x;
        if (q >= 0 && q < nx) v = x[q]; else err[0] = 2;
      }
      Bs[bk][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      const T av = As[kk + (lane >> 4)][wv * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < nblk) s1_mfma<T>(av, Bs[kk + (lane >> 4)][j * 16 + (lane & 15)], acc[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = sizeof(T) == 4 ? 4 * (lane >> 4) + v : 4 * v + (lane >> 4);
      Cs[wv * 16 + row][j * 16 + (lane & 15)] = acc[j][v];
    }
  __syncthreads();
  for (int e = tid; e < TILE * TILE; e += 256) {
    const int r = e / TILE, c = e % TILE;
    if (r >= mrows || c >= ncols) continue;
    const int4 R = ri[r], Cc = ci[c];
    const long long rp = rowpart[R.x * 4 + (Cc.y >> 2)];
    const long long so = specoff[((long long)R.z * 4 + (Cc.y & 3)) * nbe + Cc.z];
    const long long d = rp + so + (long long)R.y * nb[c] + Cc.w;
    if (rp < 0 || so < 0 || d >= nout) { err[0] = 3; continue; }
    out[d] = Cs[r][c];
  }
}

// ---------------------------------------------------------------------------
// precontracted left operator
// ---------------------------------------------------------------------------
// LW of one row block (output channel B, bra state s1', bra sector alpha'): element
// (i', k) with k in piece p (site state s1, ket sector alpha) sums the operator
// entries of (B, s1', s1) times L_A[alpha' + i'][alpha + k - pk]; the K padding is
// written as zero.  Consecutive threads take consecutive k (consecutive L columns).
__global__ __launch_bounds__(256) void lw_build_kernel(const BsLwBlock* __restrict__ blocks,
                                                       const BsLwGroup* __restrict__ groups,
                                                       const int* __restrict__ tptr, const int* __restrict__ tA,
                                                       const double* __restrict__ tv, const int* __restrict__ aoff,
                                                       const double* __restrict__ L, long long nL, int rlp,
                                                       double* __restrict__ lw, long long nlw, int* __restrict__ err) {
  const BsLwBlock b = blocks[blockIdx.x];
  const BsLwGroup& G = groups[b.g];  // read in place: its piece arrays are indexed at run time
  const long long rl2 = (long long)rlp * rlp;
  const int tot = b.n * G.K4;
  for (int e = threadIdx.x; e < tot; e += 256) {
    const int ip = e / G.K4, k = e - ip * G.K4;
    double acc = 0.0;
    if (k < G.K) {
      int p = 0;
      while (p + 1 < G.np && k >= G.pk[p + 1]) ++p;
      const int s1 = G.ps[p];
      const long long rc = (long long)(aoff[b.ap] + ip) * rlp + aoff[G.pa[p]] + (k - G.pk[p]);
      for (int t = tptr[b.bs * 4 + s1]; t < tptr[b.bs * 4 + s1 + 1]; ++t) {
        const long long q = (long long)tA[t] * rl2 + rc;
        if (q >= 0 && q < nL) acc += tv[t] * L[q]; else err[0] = 11;
      }
    }
    const long long d = G.a0 + (long long)(b.r0 + ip) * G.K4 + k;
    if (d >= 0 && d < nlw) lw[d] = acc; else err[0] = 11;
  }
}

// WR block of one panel chunk (B, s2): element (b, j') sums the operator entries of
// (B, s2', s2) times R_C[beta' + j'][beta + b] (C >= RC: the block channels Rt); rows
// b of the panel's [K][N] matrix from the chunk's column.  Consecutive threads take
// consecutive b (consecutive R columns).
__global__ __launch_bounds__(256) void wr_build_kernel(const BsWrItem* __restrict__ items,
                                                       const BsPanel* __restrict__ panels,
                                                       const int* __restrict__ tptr, const int* __restrict__ tC,
                                                       const double* __restrict__ tv, const int* __restrict__ boff,
                                                       const int* __restrict__ nbeta, const double* __restrict__ R,
                                                       long long nR, const double* __restrict__ Rt, long long nRt,
                                                       int RC, int rrp, double* __restrict__ wr, long long nwr,
                                                       int* __restrict__ err) {
  const BsWrItem it = items[blockIdx.x];
  const BsPanel P = panels[it.P];
  const int B = it.bs2 >> 2, s2 = it.bs2 & 3;
  const int nb = nbeta[it.be], np = P.N;
  const long long rr2 = (long long)rrp * rrp;
  const int ti = (B * 4 + P.s2p) * 4 + s2;
  const int t0 = tptr[ti], t1 = tptr[ti + 1];
  for (int e = threadIdx.x; e < nb * np; e += 256) {
    const int jp = e / nb, b = e - jp * nb;
    const long long rc = (long long)(boff[P.bep] + jp) * rrp + boff[it.be] + b;
    double acc = 0.0;
    for (int t = t0; t < t1; ++t) {
      const int C = tC[t];
      if (C < RC) {
        const long long q = (long long)C * rr2 + rc;
        if (q >= 0 && q < nR) acc += tv[t] * R[q]; else err[0] = 16;
      } else {
        const long long q = (long long)(C - RC) * rr2 + rc;
        if (q >= 0 && q < nRt) acc += tv[t] * Rt[q]; else err[0] = 16;
      }
    }
    const long long d = P.wbase + (long long)(it.kc + b) * np + jp;
    if (d >= 0 && d < nwr) wr[d] = acc; else err[0] = 16;
  }
}

// T2 = LW x for one tile of LW_ROWS rows of a group, all its columns (in passes of NC):
// four waves of two 16-row blocks, 16 x 16 x 4 MFMA blocks over K in slices of KS.  The
// x slice (shared by the waves) is staged in LDS with all threads loading; every lane
// reads its A fragments (one LW row, four consecutive k per MFMA step) straight from
// memory.  Results go from the accumulators to T2, where the columns of one s2 of a
// row are contiguous and the rows of one row block follow each other.
// MODE 1 writes T2 (rows (B, s2)); MODE 2 writes the chunk stores of the panels.  S is
// the storage type of LW, x and the output (T, or bfloat16 with T = float).
template <typename T, int MODE, typename S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void lw_gemm_kernel(
    const BsLwTile* __restrict__ tiles, const BsLwGroup* __restrict__ groups, const BsLwBlock* __restrict__ blocks,
    const int* __restrict__ krow, const int2* __restrict__ col, const S* __restrict__ lw, long long nlw,
    const S* __restrict__ x, long long nx, const long long* __restrict__ rowbase2,
    const long long* __restrict__ specoff, const int* __restrict__ nbeta, int nbe, const BsZeta* __restrict__ zetas,
    const int* __restrict__ kctab, S* __restrict__ out, long long nout, int* __restrict__ err) {
  constexpr int ND = 4;  // destinations per row: one per s2
  constexpr int KS = sizeof(T) == 4 ? 32 : 16;  // K slice
  constexpr int NB = sizeof(T) == 4 ? 8 : 4;    // 16-column blocks per pass
  constexpr int NC = NB * 16;
  constexpr int MB = LW_ROWS / 64;              // 16-row blocks per wave
  const BsLwTile t = tiles[blockIdx.x];
  const BsLwGroup G = groups[t.g];
  __shared__ T Bs[KS][NC + 4];
  __shared__ long long rd[LW_ROWS][ND];
  __shared__ int2 cl[NC];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int mrows = min(LW_ROWS, G.M - t.m0);
  if (MODE == 2 && tid < LW_ROWS) {
    // chunk-store offset of row (B, s1', alpha', i') for each s2: the chunk (B, s2) of the
    // zeta alpha' + q(s1'), its row (s1', alpha', i'); -1 where no panel uses the chunk
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) rd[tid][s2] = -1;
    if (tid < mrows) {
      const int r = t.m0 + tid;
      int q = -1, ip = 0;
      for (int i = 0; i < t.nrb; ++i) {
        const BsLwBlock b = blocks[t.rb0 + i];
        if (r >= b.r0 && r < b.r0 + b.n) {
          q = t.rb0 + i;
          ip = r - b.r0;
          break;
        }
      }
      if (q < 0 || blocks[q].kci < 0) {
        err[0] = 12;
      } else {
        const BsLwBlock b = blocks[q];
        const BsZeta& Z = zetas[b.zi];
        const int row = Z.row0[b.bs & 3] + ip;
        const int4 k4 = reinterpret_cast<const int4*>(kctab)[b.kci];
        const int kcs[4] = {k4.x, k4.y, k4.z, k4.w};
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int kc = kcs[s2], be = G.be[s2];
          if (kc >= 0 && be >= 0) rd[tid][s2] = Z.zbase + (long long)kc * Z.M + (long long)row * ((nbeta[be] + 7) & ~7);
          else if (be >= 0) err[0] = 12;
        }
      }
    }
  }
  if (MODE == 1 && tid < LW_ROWS) {
    // T2 offset of row (B, s1', alpha', i') for each s2: row (B, s2), spectator (alpha', s1', beta), i' n_beta
    long long d4[4] = {-1, -1, -1, -1};
    if (tid < mrows) {
      const int r = t.m0 + tid;
      int q = -1, ip = 0;
      for (int i = 0; i < t.nrb; ++i) {
        const BsLwBlock b = blocks[t.rb0 + i];
        if (r >= b.r0 && r < b.r0 + b.n) {
          q = t.rb0 + i;
          ip = r - b.r0;
          break;
        }
      }
      if (q < 0) {
        err[0] = 12;
      } else {
        const BsLwBlock b = blocks[q];
        const int ch = b.bs >> 2, s1p = b.bs & 3;
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int be = G.be[s2];
          if (be < 0) continue;
          const long long rb = rowbase2[ch * 4 + s2];
          const long long so = specoff[((long long)b.ap * 4 + s1p) * nbe + be];
          if (rb < 0 || so < 0) err[0] = 12;
          else d4[s2] = rb + so + (long long)ip * nbeta[be];
        }
      }
    }
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) rd[tid][s2] = d4[s2];
  }
  // this lane's A rows (row lane % 16 of each of the wave's row blocks)
  const S* arow[MB];
  bool aok[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int r = wv * (16 * MB) + m * 16 + (lane & 15);
    const long long a = G.a0 + (long long)(t.m0 + r) * G.K4;
    aok[m] = r < mrows && a >= 0 && a + G.K4 <= nlw;
    if (r < mrows && !aok[m]) err[0] = 13;
    arow[m] = lw + (aok[m] ? a : 0);
  }
  for (int c0 = 0; c0 < G.N; c0 += NC) {
    const int nc = min(NC, G.N - c0), nblk = (nc + 15) >> 4;
    __syncthreads();  // rd written; the previous pass is done with cl
    for (int c = tid; c < NC; c += 256) cl[c] = c < nc ? col[G.n0 + c0 + c] : make_int2(0, -1);
    T acc[MB][NB][4];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[m][j][v] = T(0);
    for (int k0 = 0; k0 < G.K4; k0 += KS) {
      __syncthreads();  // cl written; the previous slice consumed
#pragma unroll 4
      for (int e = tid; e < KS * NC; e += 256) {
        const int u = e / NC, c = e % NC, k = k0 + u;
        T v = T(0);
        if (c < nc && k < G.K) {
          const long long q = (long long)krow[G.k0 + k] + cl[c].x;
          if (q >= 0 && q < nx) v = (T)ldv(x, q); else err[0] = 14;
        }
        Bs[u][c] = v;
      }
      // The slice's K order is permuted for the matrix cores: MFMA step s sums k = g KS/4 + s
      // over the lane groups g = lane / 16, so a lane's A values for the KS/4 steps are one
      // run of consecutive k (a vector load; rows are padded to a multiple of 8, so a run is
      // either inside a row or past its end) and B reads the same permutation from LDS.
      T af[MB][KS / 4];
      const int kl = k0 + (lane >> 4) * (KS / 4);
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        if (aok[m] && kl < G.K4) {
          ldrun<KS / 4>(arow[m] + kl, af[m]);
        } else {
#pragma unroll
          for (int s = 0; s < KS / 4; ++s) af[m][s] = T(0);
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < KS / 4; ++s) {
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (j < nblk) {
            const T bv = Bs[(lane >> 4) * (KS / 4) + s][j * 16 + (lane & 15)];
#pragma unroll
            for (int m = 0; m < MB; ++m) s1_mfma<T>(af[m][s], bv, acc[m][j]);
          }
      }
    }
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < nblk) {
          const int cc = j * 16 + (lane & 15);
          const int2 ci = cl[cc];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = wv * (16 * MB) + m * 16 + (sizeof(T) == 4 ? 4 * (lane >> 4) + v : 4 * v + (lane >> 4));
            if (row >= mrows || cc >= nc) continue;
            const long long d0 = rd[row][(ci.y >> 20) % ND];
            const long long d = d0 + (ci.y & 0xfffff);
            if (d0 < 0 || d >= nout) { err[0] = 15; continue; }
            stv(out, d, acc[m][j][v]);
          }
        }
  }
}

// the bfloat16 copy of a float array (operators from FP64, x from FP32)
template <typename F>
__global__ void to_bf16_kernel(const F* __restrict__ in, uint16_t* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    stv(out, i, (float)in[i]);
}

// the FP32 copy of a precontracted operator (rounded further to bfloat16 when bf16 is set)
__global__ void operator_f32_kernel(const double* __restrict__ in, float* __restrict__ out, long long n, int bf16) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float v = (float)in[i];
    out[i] = bf16 ? bf16_round(v) : v;
  }
}

// ---------------------------------------------------------------------------
// mixes: out row r of a group = sum_e val_e * in row col_e of the same group,
// one spectator column per thread.  MODE 1 scatters into the T2 layout
// (rows (B, s2)), MODE 2 into the stage-4 panels (rows (a', s1', s2', i'),
// columns (C, j)).  Everything that depends on the column only (its
// destination offset for each of the four output site states) is formed once
// per thread; a row then costs its uniform descriptor, its input loads and one
// store.  Rows with a single operator entry (nearly all light rows, and heavy rows
// with one entry outside the GEMM) are taken four at a time so that their loads
// are in flight together.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline long long pick4(long long a0, long long a1, long long a2, long long a3, int i) {
  return i == 0 ? a0 : (i == 1 ? a1 : (i == 2 ? a2 : a3));
}

template <typename T, int MODE, bool HEAVY>
__global__ __launch_bounds__(MIX_COLS) void mix_kernel(
    const MixTile* __restrict__ tiles, const BsGroup* __restrict__ groups, const MixRow* __restrict__ rows,
    const int* __restrict__ ocol, const T* __restrict__ oval, const int4* __restrict__ spec,
    const T* __restrict__ in, long long nin, T* __restrict__ out, long long nout, int* __restrict__ err, int nbe,
    const long long* __restrict__ specoff, const int* __restrict__ bshift, const long long* __restrict__ pbase,
    const int* __restrict__ kbeta, const int* __restrict__ kstart, const int* __restrict__ nbeta, int round_bf16,
    const T* __restrict__ tmp, long long ntmp, const int* __restrict__ stage, int nstage,
    const int* __restrict__ oloc, int noloc) {
  // staged input rows [MIX_STAGE][MIX_COLS] in dynamic LDS (given only to launches that
  // stage); every thread reads back only its own column, so no barrier is needed
  extern __shared__ __align__(16) unsigned char mix_smem[];
  T(*stg)[MIX_COLS] = reinterpret_cast<T(*)[MIX_COLS]>(mix_smem);
  const MixTile t = tiles[blockIdx.x];
  const BsGroup G = groups[t.g];
  const int col = t.c0 + (int)threadIdx.x;
  if (col >= G.ncols) return;
  const bool in_lds = !HEAVY && t.ns > 0;
  if (in_lds && (t.ns > MIX_STAGE || t.s0 < 0 || t.s0 + t.ns > nstage)) {
    err[0] = 4;
    return;
  }
  int lo = 0, hi = G.nspec - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (spec[G.spec0 + mid].x <= col) lo = mid; else hi = mid - 1;
  }
  const int4 sp = spec[G.spec0 + lo];  // {start, alpha', s, beta}
  const int within = col - sp.x;
  // destination offset of this column for output site state 0..3
  // (-1: no destination, -2: inconsistent tables)
  long long c0 = -1, c1 = -1, c2 = -1, c3 = -1;
  long long stride = 0;
  if (MODE == 1) {
    const long long* so = specoff + (long long)sp.y * 4 * nbe + sp.w;
    c0 = so[0];
    c1 = so[nbe];
    c2 = so[2LL * nbe];
    c3 = so[3LL * nbe];
    c0 = c0 < 0 ? -2 : c0 + within;
    c1 = c1 < 0 ? -2 : c1 + within;
    c2 = c2 < 0 ? -2 : c2 + within;
    c3 = c3 < 0 ? -2 : c3 + within;
  } else {
    const int nb = nbeta[sp.w];
    const int wi = within / nb, wj = within - wi * nb;
    stride = nb;
    long long cz[4];
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      cz[z] = -1;
      const int cl = G.cls[z];
      if (cl < 0) continue;
      const int bp = bshift[cl * nbe + sp.w];
      if (bp < 0) continue;
      const long long pb = pbase[(((long long)sp.y * 4 + sp.z) * 4 + z) * nbe + bp];
      const int ks = kstart[(long long)bp * nbe + sp.w];
      cz[z] = (pb < 0 || ks < 0) ? -2 : pb + (long long)wi * kbeta[bp] + ks + wj;
    }
    c0 = cz[0]; c1 = cz[1]; c2 = cz[2]; c3 = cz[3];
  }
  const T* src = in + G.in_base + col;
  const long long ld = G.ld;
  const long long lim = nin - G.in_base - col;  // src[q] valid for 0 <= q < lim
  if (in_lds) {
    // eight loads in flight before their LDS stores
    for (int k0 = 0; k0 < t.ns; k0 += 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[u] = T(0);
        if (k0 + u < t.ns) {
          const long long q = (long long)stage[t.s0 + k0 + u] * ld;
          if (q >= 0 && q < lim) v[u] = src[q]; else err[0] = 4;
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + u < t.ns) stg[k0 + u][threadIdx.x] = v[u];
    }
  }
  // input value of operator entry e for this column
  auto in_at = [&](int e) -> T {
    if (in_lds) {
      const int l = e >= 0 && e < noloc ? oloc[e] : -1;
      if (l >= 0 && l < t.ns) return stg[l][threadIdx.x];
      err[0] = 4;
      return T(0);
    }
    const long long q = (long long)ocol[e] * ld;
    if (q >= 0 && q < lim) return src[q];
    err[0] = 4;
    return T(0);
  };
  auto store = [&](const MixRow& R, T v) {
    long long d;
    const long long c = pick4<T>(c0, c1, c2, c3, R.sy);
    if (MODE == 1) {
      const long long rb = pick4<T>(R.b[0], R.b[1], R.b[2], R.b[3], sp.z);
      if (rb < 0 || c < 0) { err[0] = 5; return; }
      d = rb + c;
    } else {
      if (c == -1) return;  // the output channel does not reach this column's right sector
      if (c < 0 || R.rank < 0) { err[0] = 6; return; }
      d = c + (long long)R.rank * stride;
      if (round_bf16) v = (T)bf16_round((float)v);
    }
    if (d < 0 || d >= nout) { err[0] = 7; return; }
    out[d] = v;
  };
  auto value = [&](const MixRow& R) {
    T acc = T(0);
    if (HEAVY && R.h >= 0) {
      const long long q = R.h + col;
      if (q < ntmp) acc = tmp[q]; else err[0] = 4;
    }
    for (int e = R.e0; e < R.e1; ++e) acc += oval[e] * in_at(e);
    return acc;
  };
  auto staged = [&](const MixRow& R) {
    // heavy row: the part over the shared input rows formed by the GEMM
    if (!HEAVY || R.h < 0) return T(0);
    const long long q = R.h + col;
    if (q < ntmp) return tmp[q];
    err[0] = 4;
    return T(0);
  };
  int r = t.r0;
  for (; r + 4 <= t.r1; r += 4) {
    const MixRow R0 = rows[r], R1 = rows[r + 1], R2 = rows[r + 2], R3 = rows[r + 3];
    if (R0.e1 - R0.e0 == 1 && R1.e1 - R1.e0 == 1 && R2.e1 - R2.e0 == 1 && R3.e1 - R3.e0 == 1) {
      const T v0 = in_at(R0.e0), v1 = in_at(R1.e0), v2 = in_at(R2.e0), v3 = in_at(R3.e0);
      const T h0 = staged(R0), h1 = staged(R1), h2 = staged(R2), h3 = staged(R3);
      store(R0, h0 + oval[R0.e0] * v0);
      store(R1, h1 + oval[R1.e0] * v1);
      store(R2, h2 + oval[R2.e0] * v2);
      store(R3, h3 + oval[R3.e0] * v3);
    } else {
      store(R0, value(R0));
      store(R1, value(R1));
      store(R2, value(R2));
      store(R3, value(R3));
    }
  }
  for (; r < t.r1; ++r) {
    const MixRow R = rows[r];
    store(R, value(R));
  }
}

// ---------------------------------------------------------------------------
// stage 4: partial[slot] = panel rows [m0, m0+64) x stacked R columns [n0, n0+64)
// over K in [k0, k1); the reduction sums the K chunks and writes rows of y.
// One stage-4 tile on the matrix cores: four waves of 16 panel rows each,
// 16 x 16 x 4 MFMA blocks over the (at most four) 16-column blocks that lie
// inside N, K staged through two LDS buffers (the next K slice is fetched into
// registers while the current one is multiplied).  Accumulator register v of
// lane l holds D[4*(l/16)+v][l%16] (FP32) or D[4*v+l/16][l%16] (FP64).
template <typename T>
__device__ inline void s4_mfma(T a, T b, T (&c)[4]);
template <>
__device__ inline void s4_mfma<float>(float a, float b, float (&c)[4]) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  v4 x = {c[0], c[1], c[2], c[3]};
  x = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, x, 0, 0, 0);
  c[0] = x[0]; c[1] = x[1]; c[2] = x[2]; c[3] = x[3];
}
template <>
__device__ inline void s4_mfma<double>(double a, double b, double (&c)[4]) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  v4 x = {c[0], c[1], c[2], c[3]};
  x = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, x, 0, 0, 0);
  c[0] = x[0]; c[1] = x[1]; c[2] = x[2]; c[3] = x[3];
}

template <typename T>
__global__ __launch_bounds__(256) void stage4_mfma_kernel(const BsS4Tile* __restrict__ tiles, const T* __restrict__ A,
                                                          long long nA, const T* __restrict__ B, long long nB,
                                                          T* __restrict__ part, int* __restrict__ err) {
  const BsS4Tile t = tiles[blockIdx.x];
  if (t.abase < 0 || t.abase + (long long)t.M * t.K > nA || t.bbase < 0 || t.bbase + (long long)t.K * t.N > nB) {
    if (threadIdx.x == 0) err[0] = 8;
    return;
  }
  constexpr int KS = sizeof(T) == 4 ? 32 : 16;  // K slice (two LDS buffers stay under 64 KB)
  constexpr int RUNL = KS / 4;                   // elements per thread per operand slice
  __shared__ T As[2][KS][TILE + 4];
  __shared__ T Bs[2][KS][TILE + 4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nvalid = min(TILE, t.N - t.n0);
  const int nblk = (nvalid + 15) >> 4;
  // global -> register runs: A (64 rows x KS: row tid/4, RUNL consecutive k), B (KS x 64: k tid*RUNL/64, RUNL columns)
  const int ar = tid >> 2, ak = (tid & 3) * RUNL;
  const int bk = tid / (TILE / RUNL), bn = (tid % (TILE / RUNL)) * RUNL;
  T ra[RUNL], rb[RUNL];
  auto fetch = [&](int k0) {
    const long long arow = t.abase + (long long)(t.m0 + ar) * t.K;
    const bool rowok = t.m0 + ar < t.M;
#pragma unroll
    for (int u = 0; u < RUNL; ++u) {
      const int k = k0 + ak + u;
      ra[u] = (rowok && k < t.k1) ? A[arow + k] : T(0);
    }
    const int kb = k0 + bk;
    const long long brow = t.bbase + (long long)kb * t.N + t.n0;
#pragma unroll
    for (int u = 0; u < RUNL; ++u) rb[u] = (kb < t.k1 && bn + u < nvalid) ? B[brow + bn + u] : T(0);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < RUNL; ++u) As[buf][ak + u][ar] = ra[u];
#pragma unroll
    for (int u = 0; u < RUNL; ++u) Bs[buf][bk][bn + u] = rb[u];
  };
  T acc[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[j][v] = T(0);
  int buf = 0;
  fetch(t.k0);
  stash(0);
  __syncthreads();
  for (int k0 = t.k0; k0 < t.k1; k0 += KS) {
    const bool more = k0 + KS < t.k1;
    if (more) fetch(k0 + KS);
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      const T a = As[buf][kk + (lane >> 4)][wv * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < nblk) s4_mfma<T>(a, Bs[buf][kk + (lane >> 4)][j * 16 + (lane & 15)], acc[j]);
    }
    if (more) {
      stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  // only the tile's valid rows and columns (the reduction reads no others)
  T* P = part + (long long)t.slot * (TILE * TILE);
  const int mvalid = min(TILE, t.M - t.m0);
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = sizeof(T) == 4 ? 4 * (lane >> 4) + v : 4 * v + (lane >> 4);
      if (wv * 16 + row < mvalid && j * 16 + (lane & 15) < nvalid)
        P[(wv * 16 + row) * TILE + j * 16 + (lane & 15)] = acc[j][v];
    }
}

// Panel x right operator: the stage-4 tile whose A operand, the panel (zeta, s2'), is read
// from the zeta's chunk store through the panel's column table (offset and row stride per
// aligned block of 8 columns; a thread's RUNL columns lie in one such block).
template <typename T, typename S>
__global__ __launch_bounds__(256) void panel_mfma_kernel(const BsPTile* __restrict__ tiles, const BsK8* __restrict__ k8,
                                                         long long nk8, const S* __restrict__ A, long long nA,
                                                         const S* __restrict__ B, long long nB, T* __restrict__ part,
                                                         int* __restrict__ err) {
  const BsPTile t = tiles[blockIdx.x];
  if (t.abase < 0 || t.abase >= nA || t.bbase < 0 || t.bbase + (long long)t.K * t.N > nB) {
    if (threadIdx.x == 0) err[0] = 8;
    return;
  }
  constexpr int KS = sizeof(T) == 4 ? 32 : 16;  // K slice (two LDS buffers stay under 64 KB)
  constexpr int RUNL = KS / 4;                   // elements per thread per operand slice
  __shared__ T As[2][KS][TILE + 4];
  __shared__ T Bs[2][KS][TILE + 4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nvalid = min(TILE, t.N - t.n0);
  const int nblk = (nvalid + 15) >> 4;
  // global -> register runs: A (64 rows x KS: row tid/4, RUNL consecutive k), B (KS x 64: k tid*RUNL/64, RUNL columns)
  const int ar = tid >> 2, ak = (tid & 3) * RUNL;
  const int bk = tid / (TILE / RUNL), bn = (tid % (TILE / RUNL)) * RUNL;
  T ra[RUNL], rb[RUNL];
  auto fetch = [&](int k0) {
    // this thread's RUNL columns lie in one aligned block of 8 of one chunk
    const int ka = k0 + ak;
    bool rowok = t.m0 + ar < t.M && ka < t.k1;
    long long arow = 0;
    if (rowok) {
      const long long ti = t.t8 + (ka >> 3);
      const BsK8 e = ti >= 0 && ti < nk8 ? k8[ti] : BsK8{-1, 0};
      arow = t.abase + e.off + (long long)(t.m0 + ar) * e.nb8 + (ka & 7);
      if (e.off < 0 || arow < 0 || arow + RUNL > nA) {
        err[0] = 8;
        rowok = false;
      }
    }
    // the run is 16-byte aligned and lies inside [k0, k1) or past it (chunk columns and the
    // K split are multiples of 8)
    if (rowok) {
      ldrun<RUNL>(A + arow, ra);
    } else {
#pragma unroll
      for (int u = 0; u < RUNL; ++u) ra[u] = T(0);
    }
    const int kb = k0 + bk;
    const long long brow = t.bbase + (long long)kb * t.N + t.n0;
#pragma unroll
    for (int u = 0; u < RUNL; ++u) rb[u] = (kb < t.k1 && bn + u < nvalid) ? (T)ldv(B, brow + bn + u) : T(0);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < RUNL; ++u) As[buf][ak + u][ar] = ra[u];
#pragma unroll
    for (int u = 0; u < RUNL; ++u) Bs[buf][bk][bn + u] = rb[u];
  };
  T acc[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[j][v] = T(0);
  int buf = 0;
  fetch(t.k0);
  stash(0);
  __syncthreads();
  for (int k0 = t.k0; k0 < t.k1; k0 += KS) {
    const bool more = k0 + KS < t.k1;
    if (more) fetch(k0 + KS);
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      const T a = As[buf][kk + (lane >> 4)][wv * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < nblk) s4_mfma<T>(a, Bs[buf][kk + (lane >> 4)][j * 16 + (lane & 15)], acc[j]);
    }
    if (more) {
      stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  // only the tile's valid rows and columns (the reduction reads no others)
  T* P = part + (long long)t.slot * (TILE * TILE);
  const int mvalid = min(TILE, t.M - t.m0);
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = sizeof(T) == 4 ? 4 * (lane >> 4) + v : 4 * v + (lane >> 4);
      if (wv * 16 + row < mvalid && j * 16 + (lane & 15) < nvalid)
        P[(wv * 16 + row) * TILE + j * 16 + (lane & 15)] = acc[j][v];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void reduce4_kernel(const BsRedTile* __restrict__ red, const T* __restrict__ part,
                                                      const long long* __restrict__ rowdst, T* __restrict__ y,
                                                      long long ny, int* __restrict__ err) {
  const BsRedTile t = red[blockIdx.x];
  for (int e = threadIdx.x; e < TILE * TILE; e += 256) {
    const int r = e / TILE, c = e % TILE;
    if (t.m0 + r >= t.M || t.n0 + c >= t.N) continue;
    // four partial sums in flight, combined in a fixed order (deterministic)
    const T* pp = part + (long long)t.slot0 * (TILE * TILE) + e;
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    int q = 0;
    for (; q + 4 <= t.nsplit; q += 4) {
      s0 += pp[(long long)q * (TILE * TILE)];
      s1 += pp[(long long)(q + 1) * (TILE * TILE)];
      s2 += pp[(long long)(q + 2) * (TILE * TILE)];
      s3 += pp[(long long)(q + 3) * (TILE * TILE)];
    }
    for (; q < t.nsplit; ++q) s0 += pp[(long long)q * (TILE * TILE)];
    const T s = (s0 + s1) + (s2 + s3);
    const long long d = rowdst[t.row0 + t.m0 + r] + t.n0 + c;
    if (d < 0 || d >= ny) { err[0] = 9; continue; }
    y[d] = s;
  }
}

// stacked R of sector beta': rows (C, j) with b = off(beta) + j, columns j' with b' = off(beta') + j'
template <typename T>
__global__ __launch_bounds__(256) void rstack_kernel(const BsPair* __restrict__ pairs, const int* __restrict__ boff,
                                                     const int* __restrict__ nbeta,
                                                     const long long* __restrict__ rbase, int RC, int RCx, int rrp,
                                                     const T* __restrict__ R, const T* __restrict__ Rt,
                                                     T* __restrict__ rs, long long nrs, int* __restrict__ err) {
  const BsPair p = pairs[blockIdx.x];
  const int nb = nbeta[p.beta], nbp = nbeta[p.bprime], ob = boff[p.beta], obp = boff[p.bprime];
  const long long rr2 = (long long)rrp * rrp;
  const T* src = p.C < RC ? R + (long long)p.C * rr2 : Rt + (long long)(p.C - RC) * rr2;
  T* dst = rs + rbase[p.bprime] + (long long)p.koff * nbp;
  if (p.C < 0 || p.C >= RCx || ob < 0 || obp < 0 || ob + nb > rrp || obp + nbp > rrp ||
      rbase[p.bprime] + (long long)(p.koff + nb) * nbp > nrs) {
    if (threadIdx.x == 0) err[0] = 10;
    return;
  }
  for (int e = threadIdx.x; e < nb * nbp; e += 256) {
    const int j = e / nbp, jp = e - j * nbp;
    dst[(long long)j * nbp + jp] = src[(long long)(obp + jp) * rrp + ob + j];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
static void build_mix(Engine& E, BsMix& m, int mode, const SiteOp& so, const std::vector<Q2>& dout, int nout_ch,
                      const std::vector<int>& rowidx_in, const std::vector<int>& grp_in, const std::map<Q2, int>& gid,
                      const std::vector<Q2>& gq, const std::vector<int>& cols, const std::vector<int>& ldg,
                      const std::vector<long long>& in_off, const std::vector<int>& nrows_in,
                      const std::vector<int>& nshared, const std::vector<int>& spec0, const std::vector<int>& nspec,
                      const std::vector<long long>& rowbase2, const std::vector<int>& crank,
                      const std::vector<std::array<int, 4>>& gcls) {
  const int ng = (int)gq.size();
  std::vector<std::vector<int2>> rows_by_g(ng);
  for (int K = 0; K < nout_ch; ++K)
    for (int s = 0; s < 4; ++s) {
      auto it = gid.find(sub(kSiteQ[s], dout[K]));
      if (it != gid.end()) rows_by_g[it->second].push_back(make_int2(K, s));
    }
  auto descriptor = [&](int2 ro, int e0, int e1, long long h) {
    MixRow R{};
    R.e0 = e0;
    R.e1 = e1;
    R.h = h;
    R.sy = ro.y;
    for (int z = 0; z < 4; ++z) R.b[z] = mode == 1 ? rowbase2[(size_t)ro.x * 4 + z] : -1;
    R.rank = mode == 2 ? crank[ro.x] : 0;
    return R;
  };
  std::vector<int> ocol;
  std::vector<double> oval;
  std::vector<MixRow> lrows, hrows_all;
  std::vector<MixTile> tiles;
  std::vector<BsGroup> groups(ng);
  std::vector<MixTile> htiles;
  std::vector<int> stage;  // staged input rows of the light tiles
  std::vector<int> oloc;   // per operator entry: its input row's position in its tile's staged list
  std::vector<double> hw;
  m.heavy.clear();
  m.ntmp = 0;
  m.nstaged = 0;
  m.flops = m.nin = m.nout = 0.0;
  m.fl_light = m.el_light = m.fl_heavy = m.el_heavy = m.el_scatter = 0.0;
  for (int g = 0; g < ng; ++g) {
    groups[g] = BsGroup{in_off[g], cols[g], spec0[g], nspec[g], ldg[g], {gcls[g][0], gcls[g][1], gcls[g][2], gcls[g][3]}};
    long long nnz_g = 0;
    std::vector<std::pair<int, double>> ent;
    std::vector<std::vector<std::pair<int, double>>> hrows, multi;
    std::vector<int2> hro, mro;
    const int r0 = (int)lrows.size();
    for (const int2& ro : rows_by_g[g]) {
      const int K = ro.x, sp = ro.y;
      ent.clear();
      for (int e = so.hptr[K]; e < so.hptr[K + 1]; ++e) {
        const int A = so.hsrc[e];
        for (int s = 0; s < 4; ++s) {
          const double v = so.hop[(size_t)e * 16 + sp * 4 + s];
          if (v == 0.0) continue;
          const int ri = rowidx_in[A * 4 + s];
          if (ri < 0 || grp_in[A * 4 + s] != g)
            throw std::runtime_error("block-sparse plan: MPO entry breaks the charge grouping");
          ent.emplace_back(ri, v);
        }
      }
      if ((int)ent.size() > HEAVY_MIN) {
        hrows.push_back(ent);
        hro.push_back(ro);
      } else if (ent.size() != 1) {
        // several entries, or none (the output row is written as zero)
        multi.push_back(ent);
        mro.push_back(ro);
      } else {
        // single-entry rows first: the kernel takes them four at a time
        lrows.push_back(descriptor(ro, (int)ocol.size(), (int)ocol.size() + 1, -1));
        ocol.push_back(ent[0].first);
        oval.push_back(ent[0].second);
        nnz_g += 1;
      }
    }
    for (size_t i = 0; i < multi.size(); ++i) {
      lrows.push_back(descriptor(mro[i], (int)ocol.size(), (int)(ocol.size() + multi[i].size()), -1));
      for (auto& pv : multi[i]) {
        ocol.push_back(pv.first);
        oval.push_back(pv.second);
      }
      nnz_g += (long long)multi[i].size();
    }
    const int r1 = (int)lrows.size();
    if (cols[g] == 0) continue;
    m.nin += (double)nrows_in[g] * cols[g];
    m.nout += (double)(r1 - r0 + (int)hro.size()) * cols[g];
    m.flops += 2.0 * (double)nnz_g * cols[g];
    if (r1 > r0) {
      m.fl_light += 2.0 * (double)nnz_g * cols[g];
      m.el_light += (double)(nrows_in[g] + (r1 - r0)) * cols[g];
    }
    if (r1 > r0) {
      // Rows whose operator entries re-read the same input rows (many more entries than
      // distinct inputs over the group) are cut into chunks whose distinct inputs fit the
      // LDS stage; each chunk's inputs are then read once per column instead of once per
      // entry.  Groups without that reuse keep direct reads in chunks of MIX_ROWS rows.
      long long nent = 0;
      std::vector<int> dist;
      for (int r = r0; r < r1; ++r)
        for (int e = lrows[r].e0; e < lrows[r].e1; ++e) {
          dist.push_back(ocol[e]);
          ++nent;
        }
      std::sort(dist.begin(), dist.end());
      dist.erase(std::unique(dist.begin(), dist.end()), dist.end());
      const int policy = E.opts.mix_stage;
      const bool use_stage = nent > 0 && (policy == 1 || (policy == 0 && (double)nent >= 1.5 * (double)dist.size()));
      oloc.resize(ocol.size(), -1);  // the group's light-row entries are all in ocol by now
      std::vector<std::array<int, 4>> chunks;  // r0, r1, s0, ns
      if (!use_stage) {
        for (int q0 = r0; q0 < r1; q0 += MIX_ROWS) chunks.push_back({q0, std::min(q0 + MIX_ROWS, r1), 0, 0});
      } else {
        int q = r0;
        std::vector<int> cur, nxt;
        while (q < r1) {
          cur.clear();
          int q1 = q;
          while (q1 < r1 && q1 - q < MIX_ROWS) {
            nxt = cur;
            for (int e = lrows[q1].e0; e < lrows[q1].e1; ++e) nxt.push_back(ocol[e]);
            std::sort(nxt.begin(), nxt.end());
            nxt.erase(std::unique(nxt.begin(), nxt.end()), nxt.end());
            if ((int)nxt.size() > MIX_STAGE && q1 > q) break;
            cur.swap(nxt);
            ++q1;
          }
          if ((int)cur.size() > MIX_STAGE)
            throw std::runtime_error("block-sparse plan: a light row reads more input rows than the mix stage holds");
          const int s0 = (int)stage.size();
          stage.insert(stage.end(), cur.begin(), cur.end());
          for (int r = q; r < q1; ++r)
            for (int e = lrows[r].e0; e < lrows[r].e1; ++e)
              oloc[e] = (int)(std::lower_bound(cur.begin(), cur.end(), ocol[e]) - cur.begin());
          chunks.push_back({q, q1, s0, (int)cur.size()});
          q = q1;
        }
      }
      for (int c0 = 0; c0 < cols[g]; c0 += MIX_COLS)
        for (const auto& ch : chunks) {
          tiles.push_back(MixTile{g, c0, ch[0], ch[1], ch[2], ch[3], 0, 0});
          m.nstaged += ch[3] > 0;
        }
    }
    if (!hro.empty()) {
      // GEMM over the group's shared input rows [0, Kd); the other entries of a heavy
      // row are added by the scatter pass
      const int h0 = (int)hrows_all.size();
      const int H = (int)hro.size(), Nin = nrows_in[g];
      // split only where it is cheaper (per spectator column: GEMM flops at ~50 TFLOP/s
      // against gathered bytes at ~1 TB/s); else the GEMM runs over the whole group
      long long nres_split = 0;
      for (int i = 0; i < H; ++i)
        for (auto& pv : hrows[i]) nres_split += pv.first >= nshared[g];
      const double cost_full = 2.0 * H * Nin / 5e13;
      const double cost_split = 2.0 * H * nshared[g] / 5e13 + 4.0 * (double)nres_split / 1e12;
      const int Kd = cost_split < cost_full ? nshared[g] : Nin, Kd4 = (Kd + 3) / 4 * 4;
      BsHeavy hv{g, H, Kd, Kd4, cols[g], ldg[g], in_off[g], (long long)hw.size(), m.ntmp};
      hw.resize(hw.size() + (size_t)H * Kd4, 0.0);
      long long nres = 0;
      // rows with exactly one entry outside the GEMM first (the scatter takes them in fours)
      std::vector<int> ord(H);
      std::iota(ord.begin(), ord.end(), 0);
      auto nout_of = [&](int i) {
        int c = 0;
        for (auto& pv : hrows[i]) c += pv.first >= Kd;
        return c;
      };
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return (nout_of(x) != 1) < (nout_of(y) != 1); });
      for (int i = 0; i < H; ++i) {
        const int hi = ord[i];
        const int e0 = (int)ocol.size();
        for (auto& pv : hrows[hi]) {
          if (pv.first < Kd) {
            hw[(size_t)hv.w_off + (size_t)i * Kd4 + pv.first] += pv.second;
          } else {
            ocol.push_back(pv.first);
            oval.push_back(pv.second);
          }
        }
        nres += (long long)ocol.size() - e0;
        hrows_all.push_back(descriptor(hro[hi], e0, (int)ocol.size(), Kd > 0 ? m.ntmp + (long long)i * ldg[g] : -1));
      }
      if (Kd > 0) m.ntmp += (long long)H * ldg[g];
      m.flops += 2.0 * ((double)H * Kd + (double)nres) * cols[g];
      m.fl_heavy += 2.0 * (double)H * Kd * cols[g];
      m.el_heavy += (double)H * Kd + (double)Kd * cols[g] + (double)H * cols[g];
      m.el_scatter += (2.0 * H + (double)nres) * cols[g];
      if (Kd > 0) m.heavy.push_back(hv);
      const int q1 = (int)hrows_all.size();
      for (int c0 = 0; c0 < cols[g]; c0 += MIX_COLS)
        for (int q0 = h0; q0 < q1; q0 += MIX_ROWS)
          htiles.push_back(MixTile{g, c0, q0, std::min(q0 + MIX_ROWS, q1), 0, 0, 0, 0});
    }
  }
  if (ocol.empty()) { ocol.push_back(0); oval.push_back(0.0); }
  oloc.resize(ocol.size(), -1);
  if (stage.empty()) stage.push_back(0);
  if (lrows.empty()) lrows.push_back(MixRow{});
  if (hrows_all.empty()) hrows_all.push_back(MixRow{});
  if (hw.empty()) hw.push_back(0.0);
  std::vector<float> oval32(oval.begin(), oval.end());
  std::vector<float> hw32(hw.begin(), hw.end());
  m.ntiles = (int)tiles.size();
  m.nhtiles = (int)htiles.size();
  hipStream_t s = E.stream;
  up(m.tiles, tiles, s);
  up(m.groups, groups, s);
  up(m.rows, lrows, s);
  up(m.ocol, ocol, s);
  up(m.stage, stage, s);
  up(m.oloc, oloc, s);
  m.nstage = (int)stage.size();
  m.noloc = (int)oloc.size();
  up(m.oval64, oval, s);
  up(m.oval32, oval32, s);
  if (!htiles.empty()) up(m.htiles, htiles, s);
  up(m.hrows, hrows_all, s);
  up(m.hw64, hw, s);
  up(m.hw32, hw32, s);
}

bool bs_build(Engine& E, BsPlan& p, int b, const Labels& ql, const Labels& qr, int rlp, int rrp, int RAx, int nP) {
  p.ok = false;
  Sectors SA, SB;
  if (!make_sectors(ql, SA) || !make_sectors(qr, SB)) return false;
  const SiteMPO& s1 = E.mpo[b];
  const SiteMPO& s2 = E.mpo[b + 1];
  const SiteOp& w1 = s1.has_block ? s1.byB_left : s1.byB;
  const SiteOp& w2 = s2.has_block ? s2.byB_rightv : s2.byB;
  const int nal = (int)SA.q.size(), nbe = (int)SB.q.size();
  const int RB = s1.Rr, RC = s2.Rr, RCx = RC + (s2.has_block ? nP : 0);
  if (w1.nout != RB || w2.nout != RCx) throw std::runtime_error("block-sparse plan: channel count mismatch");
  p.rlp = rlp; p.rrp = rrp; p.nal = nal; p.nbe = nbe; p.RAx = RAx; p.RB = RB; p.RC = RC; p.RCx = RCx;
  // channel charges (virtual channels carry the charge of the block channel they stand for)
  std::vector<Q2> dA(RAx), dB(RB), dC(RCx);
  for (int A = 0; A < RAx; ++A) dA[A] = A < s1.Rl ? E.chan_q[b][A] : E.chan_q[b + 1][s1.q0 + (A - s1.Rl)];
  for (int B = 0; B < RB; ++B) dB[B] = E.chan_q[b + 1][B];
  for (int C = 0; C < RCx; ++C) dC[C] = C < RC ? E.chan_q[b + 2][C] : E.chan_q[b + 1][s2.p0 + (C - RC)];

  // spectator groups
  std::map<Q2, int> gid;
  std::vector<Q2> gq;
  std::vector<int> cols;
  std::vector<std::vector<int4>> spec_g;
  std::vector<long long> specoff((size_t)nal * 4 * nbe, -1);
  for (int a = 0; a < nal; ++a)
    for (int s = 0; s < 4; ++s)
      for (int be = 0; be < nbe; ++be) {
        const Q2 G = sub(sub(SB.q[be], SA.q[a]), kSiteQ[s]);
        auto it = gid.find(G);
        int g;
        if (it == gid.end()) {
          g = (int)gq.size();
          gid[G] = g;
          gq.push_back(G);
          cols.push_back(0);
          spec_g.emplace_back();
        } else {
          g = it->second;
        }
        specoff[((size_t)a * 4 + s) * nbe + be] = cols[g];
        spec_g[g].push_back(make_int4(cols[g], a, s, be));
        cols[g] += SA.n[a] * SB.n[be];
      }
  const int ng = (int)gq.size();
  std::vector<int4> spec;
  std::vector<int> spec0(ng), nspec(ng);
  for (int g = 0; g < ng; ++g) {
    spec0[g] = (int)spec.size();
    nspec[g] = (int)spec_g[g].size();
    spec.insert(spec.end(), spec_g[g].begin(), spec_g[g].end());
  }

  // Inputs shared by the heavy rows of a mix: an output row with more than HEAVY_MIN
  // operator entries goes through a dense GEMM, but its entries typically split into
  // a few input rows common to most heavy rows of the group and one or two of its
  // own.  The common input rows are stored first in their group so that the GEMM
  // runs over them only; the remaining entries are added by the scatter pass.
  auto shared_inputs = [&](const SiteOp& so, const std::vector<Q2>& dout, int nout_ch, int nin_ch) {
    std::vector<int> cnt((size_t)nin_ch * 4, 0), heavy(ng, 0);
    std::vector<int> ent;
    for (int K = 0; K < nout_ch; ++K)
      for (int sp = 0; sp < 4; ++sp) {
        if (gid.find(sub(kSiteQ[sp], dout[K])) == gid.end()) continue;
        ent.clear();
        for (int e = so.hptr[K]; e < so.hptr[K + 1]; ++e)
          for (int s = 0; s < 4; ++s)
            if (so.hop[(size_t)e * 16 + sp * 4 + s] != 0.0) ent.push_back(so.hsrc[e] * 4 + s);
        if ((int)ent.size() <= HEAVY_MIN) continue;
        ++heavy[gid.find(sub(kSiteQ[sp], dout[K]))->second];
        for (int id : ent) ++cnt[id];
      }
    return std::make_pair(cnt, heavy);
  };
  // row grouping of T1 (rows (A, s1)) and T2 (rows (B, s2)); shared heavy inputs first
  auto rows_of = [&](const std::vector<Q2>& d, int n, const std::vector<int>& cnt, const std::vector<int>& heavy,
                     std::vector<int>& idx, std::vector<int>& grp, std::vector<int>& nrows, std::vector<int>& nshared) {
    idx.assign((size_t)n * 4, -1);
    grp.assign((size_t)n * 4, -1);
    nrows.assign(ng, 0);
    nshared.assign(ng, 0);
    std::vector<char> sh((size_t)n * 4, 0);
    for (int K = 0; K < n; ++K)
      for (int s = 0; s < 4; ++s) {
        auto it = gid.find(sub(kSiteQ[s], d[K]));
        if (it == gid.end()) continue;
        grp[K * 4 + s] = it->second;
        const int H = heavy[it->second];
        sh[K * 4 + s] = H > 0 && cnt[K * 4 + s] >= std::max(4, H / 16);
      }
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < n * 4; ++i) {
        if (grp[i] < 0 || (sh[i] != 0) != (pass == 0)) continue;
        idx[i] = nrows[grp[i]]++;
        if (pass == 0) ++nshared[grp[i]];
      }
  };
  auto u1 = shared_inputs(w1, dB, RB, RAx);
  auto u2 = shared_inputs(w2, dC, RCx, RB);
  std::vector<int> idx1, grp1, nr1, idx2, grp2, nr2, ns1, ns2;
  rows_of(dA, RAx, u1.first, u1.second, idx1, grp1, nr1, ns1);
  rows_of(dB, RB, u2.first, u2.second, idx2, grp2, nr2, ns2);
  // group rows are stored with a stride rounded up to 4 elements (16-byte aligned rows)
  std::vector<int> ldg(ng);
  for (int g = 0; g < ng; ++g) ldg[g] = (cols[g] + 3) / 4 * 4;
  std::vector<long long> off1(ng), off2(ng);
  long long n1 = 0, n2 = 0;
  for (int g = 0; g < ng; ++g) {
    off1[g] = n1; n1 += (long long)nr1[g] * ldg[g];
    off2[g] = n2; n2 += (long long)nr2[g] * ldg[g];
  }
  std::vector<long long> rowpart1((size_t)RAx * 4, -1), rowbase2((size_t)RB * 4, -1);
  for (int i = 0; i < RAx * 4; ++i)
    if (idx1[i] >= 0) rowpart1[i] = off1[grp1[i]] + (long long)idx1[i] * ldg[grp1[i]];
  for (int i = 0; i < RB * 4; ++i)
    if (idx2[i] >= 0) rowbase2[i] = off2[grp2[i]] + (long long)idx2[i] * ldg[grp2[i]];
  p.n1 = n1;
  p.n2 = n2;

  // precontracted left operator: row blocks (B, s1', alpha') grouped by (gamma, mask)
  p.lw = E.opts.precontract >= 1 && (long long)rlp * 16 * rrp < (1LL << 31);
  p.wr = p.lw && E.opts.precontract == 2;
  p.build_wr = 0.0;
  p.nwr = p.nk8 = 0;
  p.npanels = p.nwr_items = p.nptiles = 0;
  p.have_lw64 = p.have_lw16 = p.have_wr16 = false;
  p.lw32_state = p.wr32_state = 0;
  // panel GEMM tables (right operator)
  std::vector<BsPTile> wptiles;
  std::vector<BsK8> wk8;
  std::vector<BsRedTile> wred;
  std::vector<long long> wrowdst;
  int wslots = 0;
  double wflops = 0.0, wbytes = 0.0, wel_red = 0.0;
  if (p.lw) {
    p.n1 = 0;
    // operator entries of (B, s1', s1): channel A and value; the charge of A is fixed by them
    std::vector<int> tptr((size_t)RB * 16 + 1, 0), tA;
    std::vector<double> tv;
    for (int B = 0; B < RB; ++B)
      for (int sp = 0; sp < 4; ++sp)
        for (int s1_ = 0; s1_ < 4; ++s1_) {
          tptr[(size_t)(B * 4 + sp) * 4 + s1_] = (int)tA.size();
          const Q2 want = add(sub(dB[B], kSiteQ[sp]), kSiteQ[s1_]);  // d_A = d_B + q(s1) - q(s1')
          for (int e = w1.hptr[B]; e < w1.hptr[B + 1]; ++e) {
            const double v = w1.hop[(size_t)e * 16 + sp * 4 + s1_];
            if (v == 0.0) continue;
            if (dA[w1.hsrc[e]] != want)
              throw std::runtime_error("block-sparse plan: MPO entry breaks the charge grouping");
            tA.push_back(w1.hsrc[e]);
            tv.push_back(v);
          }
        }
    tptr[(size_t)RB * 16] = (int)tA.size();
    const QLook fa(SA), fb(SB);
    // right operator: panels (zeta, s2') and their chunks (B, s2), WR blocks, chunk table
    std::map<Q2, int> zid;
    std::vector<Q2> zq;
    std::vector<BsZeta> zetas;
    std::vector<BsPanel> panels;
    std::vector<BsWrItem> items;
    std::vector<int> kctab, bzk, t2ptr, t2C;
    std::vector<double> t2v;
    if (p.wr) {
      // operator entries of the second site by (B, s2', s2): channel C and value
      std::vector<std::vector<std::pair<int, double>>> lst((size_t)RB * 16);
      for (int C = 0; C < RCx; ++C)
        for (int e = w2.hptr[C]; e < w2.hptr[C + 1]; ++e) {
          const int B = w2.hsrc[e];
          for (int s2p = 0; s2p < 4; ++s2p)
            for (int s2_ = 0; s2_ < 4; ++s2_) {
              const double v = w2.hop[(size_t)e * 16 + s2p * 4 + s2_];
              if (v == 0.0) continue;
              if (dC[C] != add(sub(dB[B], kSiteQ[s2_]), kSiteQ[s2p]))  // d_C = d_B + q(s2') - q(s2)
                throw std::runtime_error("block-sparse plan: MPO entry breaks the charge grouping");
              lst[(size_t)(B * 4 + s2p) * 4 + s2_].emplace_back(C, v);
            }
        }
      std::vector<int> rel((size_t)RB * 4, 0);  // s2' reached by the entries of (B, s2)
      t2ptr.assign((size_t)RB * 16 + 1, 0);
      for (size_t i = 0; i < lst.size(); ++i) {
        t2ptr[i] = (int)t2C.size();
        for (auto& cv : lst[i]) {
          t2C.push_back(cv.first);
          t2v.push_back(cv.second);
        }
        if (!lst[i].empty()) rel[(i / 16) * 4 + (i % 4)] |= 1 << ((i / 4) % 4);
      }
      t2ptr[(size_t)RB * 16] = (int)t2C.size();
      for (int ap = 0; ap < nal; ++ap)
        for (int sp = 0; sp < 4; ++sp) {
          const Q2 z = add(SA.q[ap], kSiteQ[sp]);
          if (!zid.count(z)) {
            zid[z] = (int)zq.size();
            zq.push_back(z);
          }
        }
      const int nz = (int)zq.size();
      zetas.resize(nz);
      bzk.assign((size_t)RB * nz, -1);
      long long npan = 0, nw = 0;
      std::vector<int> ckc;  // chunk-store column of each chunk of the current zeta
      std::vector<int2> cch;  // its (B * 4 + s2, right sector)
      for (int zi = 0; zi < nz; ++zi) {
        BsZeta& Z = zetas[zi];
        int M = 0;
        for (int sp = 0; sp < 4; ++sp) {
          const int ap = fa(sub(zq[zi], kSiteQ[sp]));
          Z.row0[sp] = ap >= 0 ? M : -1;
          if (ap >= 0) M += SA.n[ap];
        }
        Z.M = M;
        Z.zbase = npan;
        if (M == 0) continue;
        // the zeta's store: every chunk (B, s2) that reaches some s2' with a right sector
        ckc.clear();
        cch.clear();
        int KU = 0;
        for (int s2_ = 0; s2_ < 4; ++s2_)
          for (int B = 0; B < RB; ++B) {
            int reach = rel[(size_t)B * 4 + s2_];
            for (int s2p = 0; s2p < 4; ++s2p)
              if (fb(add(zq[zi], kSiteQ[s2p])) < 0) reach &= ~(1 << s2p);
            if (reach == 0) continue;
            const int be = fb(add(sub(zq[zi], dB[B]), kSiteQ[s2_]));
            if (be < 0) continue;
            int& kci = bzk[(size_t)B * nz + zi];
            if (kci < 0) {
              kci = (int)(kctab.size() / 4);
              kctab.resize(kctab.size() + 4, -1);
            }
            kctab[(size_t)kci * 4 + s2_] = KU;
            ckc.push_back(KU);
            cch.push_back(make_int2(B * 4 + s2_, be));
            KU += (SB.n[be] + 7) & ~7;
          }
        if ((long long)M * KU >= (1LL << 31))
          throw std::runtime_error("block-sparse plan: chunk store larger than 2^31 elements");
        for (int s2p = 0; s2p < 4; ++s2p) {
          const int bep = fb(add(zq[zi], kSiteQ[s2p]));
          if (bep < 0) continue;
          const int P = (int)panels.size();
          const size_t it0 = items.size();
          const long long t8 = (long long)wk8.size();
          int K = 0, Kr = 0;  // panel columns with and without the padding of the chunks
          for (size_t c = 0; c < ckc.size(); ++c) {
            const int bs2 = cch[c].x, be = cch[c].y;
            if (!(rel[(size_t)bs2] >> s2p & 1)) continue;
            const int nb8 = (SB.n[be] + 7) & ~7;
            items.push_back(BsWrItem{P, bs2, K, be});
            for (int c8 = 0; c8 < nb8; c8 += 8) wk8.push_back(BsK8{ckc[c] * M + c8, nb8});
            K += nb8;
            Kr += SB.n[be];
          }
          if (K == 0) continue;
          const int N = SB.n[bep];
          const int row0 = (int)wrowdst.size();
          for (int sp = 0; sp < 4; ++sp) {
            const int ap = fa(sub(zq[zi], kSiteQ[sp]));
            if (ap < 0) continue;
            for (int i = 0; i < SA.n[ap]; ++i)
              wrowdst.push_back((long long)(SA.off[ap] + i) * 16 * rrp + (long long)(sp * 4 + s2p) * rrp + SB.off[bep]);
          }
          panels.push_back(BsPanel{npan, nw, M, K, N, zi, s2p, bep, 0, 0});
          for (size_t i = it0; i < items.size(); ++i) {
            const int B = items[i].bs2 >> 2, s2_ = items[i].bs2 & 3, ti = (B * 4 + s2p) * 4 + s2_;
            p.build_wr += (double)SB.n[items[i].be] * N * (t2ptr[ti + 1] - t2ptr[ti]);
          }
          // split-K tiles of the panel product (the stage-4 kernels), rows scattered into y
          for (int m0 = 0; m0 < M; m0 += TILE)
            for (int n0 = 0; n0 < N; n0 += TILE) {
              BsRedTile r{M, N, m0, n0, wslots, 0, row0, 0};
              for (int k0 = 0; k0 < K; k0 += KSPLIT) {
                wptiles.push_back(BsPTile{npan, nw, t8, M, N, K, m0, n0, k0, std::min(K, k0 + KSPLIT), wslots});
                ++wslots;
                ++r.nsplit;
              }
              wel_red += (double)(r.nsplit + 1) * std::min(TILE, M - m0) * std::min(TILE, N - n0);
              wred.push_back(r);
            }
          wflops += 2.0 * M * (double)Kr * N;
          wbytes += (double)M * Kr + (double)Kr * N + (double)M * N;
          nw += (long long)K * N;
        }
        npan += (long long)M * KU;
      }
      p.n2 = npan;
      p.nwr = nw;
      p.npanels = (int)panels.size();
      p.nwr_items = (int)items.size();
      p.nptiles = (int)wptiles.size();
    }
    struct LwKey {
      Q2 g;
      int mask, cmask;
      bool operator<(const LwKey& o) const {
        return g != o.g ? g < o.g : (mask != o.mask ? mask < o.mask : cmask < o.cmask);
      }
    };
    std::map<LwKey, std::vector<BsLwBlock>> byg;
    for (int B = 0; B < RB; ++B)
      for (int sp = 0; sp < 4; ++sp)
        for (int ap = 0; ap < nal; ++ap) {
          const Q2 gam = sub(add(SA.q[ap], kSiteQ[sp]), dB[B]);
          // columns: the s2 whose right sector exists (and, with panels, that a panel uses)
          int cmask = 0, zi = -1, kci = -1;
          if (p.wr) {
            zi = zid.at(add(SA.q[ap], kSiteQ[sp]));
            kci = bzk[(size_t)B * zq.size() + zi];
            if (kci < 0) continue;
            for (int s2_ = 0; s2_ < 4; ++s2_)
              if (kctab[(size_t)kci * 4 + s2_] >= 0) cmask |= 1 << s2_;
          } else {
            for (int s2_ = 0; s2_ < 4; ++s2_)
              if (fb(add(gam, kSiteQ[s2_])) >= 0) cmask |= 1 << s2_;
          }
          if (cmask == 0) continue;
          int mask = 0;
          for (int s1_ = 0; s1_ < 4; ++s1_) {
            const size_t ti = (size_t)(B * 4 + sp) * 4 + s1_;
            if (fa(sub(gam, kSiteQ[s1_])) >= 0 && tptr[ti + 1] > tptr[ti]) mask |= 1 << s1_;
          }
          // no operator entry: these outputs stay zero
          if (mask == 0) continue;
          byg[LwKey{gam, mask, cmask}].push_back(BsLwBlock{0, 0, SA.n[ap], B * 4 + sp, ap, zi, kci, 0});
        }
    std::vector<BsLwGroup> lgroups;
    std::vector<BsLwBlock> blocks;
    std::vector<BsLwTile> ltiles;
    std::vector<int> krow;
    std::vector<int2> lcol;
    long long a0 = 0;
    p.flops_lw = p.bytes_lw = p.build_lw = 0.0;
    for (auto& kv : byg) {
      const Q2 gam = kv.first.g;
      BsLwGroup G{};
      G.a0 = a0;
      G.k0 = (int)krow.size();
      G.n0 = (int)lcol.size();
      G.np = 0;
      for (int s1_ = 0; s1_ < 4; ++s1_) {
        if (!(kv.first.mask >> s1_ & 1)) continue;
        const int al = fa(sub(gam, kSiteQ[s1_]));
        G.ps[G.np] = s1_;
        G.pk[G.np] = G.K;
        G.pn[G.np] = SA.n[al];
        G.pa[G.np] = al;
        ++G.np;
        for (int a = 0; a < SA.n[al]; ++a) krow.push_back((SA.off[al] + a) * 16 * rrp + s1_ * 4 * rrp);
        G.K += SA.n[al];
      }
      G.K4 = (G.K + 7) / 8 * 8;  // row stride: K rounded up to 8 (runs of 8 consecutive k per lane)
      for (int s2_ = 0; s2_ < 4; ++s2_) {
        const int be = kv.first.cmask >> s2_ & 1 ? fb(add(gam, kSiteQ[s2_])) : -1;
        G.be[s2_] = be;
        if (be < 0) continue;
        for (int j = 0; j < SB.n[be]; ++j) lcol.push_back(make_int2(s2_ * rrp + SB.off[be] + j, (s2_ << 20) | j));
        G.N += SB.n[be];
      }
      G.rb0 = (int)blocks.size();
      const int g = (int)lgroups.size();
      for (BsLwBlock& b : kv.second) {
        b.g = g;
        b.r0 = G.M;
        G.M += b.n;
        // forming LW: one multiply-add per element of the block and operator entry
        for (int q = 0; q < G.np; ++q) {
          const size_t ti = (size_t)b.bs * 4 + G.ps[q];
          p.build_lw += (double)b.n * G.pn[q] * (tptr[ti + 1] - tptr[ti]);
        }
        blocks.push_back(b);
      }
      G.nrb = (int)blocks.size() - G.rb0;
      for (int m0 = 0, i = G.rb0; m0 < G.M; m0 += LW_ROWS) {
        while (blocks[i].r0 + blocks[i].n <= m0) ++i;
        int j = i;
        while (j < G.rb0 + G.nrb && blocks[j].r0 < m0 + LW_ROWS) ++j;
        ltiles.push_back(BsLwTile{g, m0, i, j - i});
      }
      a0 += (long long)G.M * G.K4;
      p.flops_lw += 2.0 * G.M * (double)G.K * G.N;
      p.bytes_lw += (double)G.M * G.K + (double)G.K * G.N + (double)G.M * G.N;
      lgroups.push_back(G);
    }
    p.nlw = a0;
    p.nlw_groups = (int)lgroups.size();
    p.nlw_blocks = (int)blocks.size();
    p.nlw_tiles = (int)ltiles.size();
    if (krow.empty()) krow.push_back(0);
    if (lcol.empty()) lcol.push_back(make_int2(0, 0));
    if (tA.empty()) { tA.push_back(0); tv.push_back(0.0); }
    hipStream_t s0 = E.stream;
    up(p.lw_groups, lgroups, s0);
    up(p.lw_blocks, blocks, s0);
    up(p.lw_tiles, ltiles, s0);
    up(p.lw_krow, krow, s0);
    up(p.lw_col, lcol, s0);
    up(p.lw_tptr, tptr, s0);
    up(p.lw_tA, tA, s0);
    up(p.lw_tv, tv, s0);
    up(p.rowbase2, rowbase2, s0);
    up(p.aoff, SA.off, s0);
    if (p.wr) {
      if (zetas.empty()) zetas.push_back(BsZeta{});
      if (kctab.empty()) kctab.assign(4, -1);
      if (panels.empty()) panels.push_back(BsPanel{});
      if (items.empty()) items.push_back(BsWrItem{});
      if (t2C.empty()) { t2C.push_back(0); t2v.push_back(0.0); }
      up(p.lw_zeta, zetas, s0);
      up(p.lw_kc, kctab, s0);
      up(p.wr_panels, panels, s0);
      up(p.wr_items, items, s0);
      up(p.wr_tptr, t2ptr, s0);
      up(p.wr_tC, t2C, s0);
      up(p.wr_tv, t2v, s0);
      if (wk8.empty()) wk8.push_back(BsK8{0, 8});
      if (wptiles.empty()) wptiles.push_back(BsPTile{});
      p.nk8 = (long long)wk8.size();
      up(p.wr_k8, wk8, s0);
      up(p.wr_ptiles, wptiles, s0);
    }
  }

  // stage 1 tables
  std::vector<BsAlpha> alpha(nal);
  std::vector<long long> rsrc;
  std::vector<int4> rinfo, cinfo, tiles1;
  const long long rl2 = (long long)rlp * rlp;
  p.flops1 = 0.0;
  p.bytes1 = 0.0;
  for (int a = 0; a < (p.lw ? 0 : nal); ++a) {
    BsAlpha& A_ = alpha[a];
    A_.row0 = (int)rinfo.size();
    A_.col0 = (int)cinfo.size();
    A_.K = SA.n[a];
    A_.oal = SA.off[a];
    for (int A = 0; A < RAx; ++A) {
      const int ap = SA.find(add(SA.q[a], dA[A]));
      if (ap < 0) continue;
      for (int i = 0; i < SA.n[ap]; ++i) {
        rsrc.push_back((long long)A * rl2 + (long long)(SA.off[ap] + i) * rlp + SA.off[a]);
        rinfo.push_back(make_int4(A, i, ap, 0));
      }
    }
    for (int s1_ = 0; s1_ < 4; ++s1_)
      for (int s2_ = 0; s2_ < 4; ++s2_) {
        const int be = SB.find(add(add(SA.q[a], kSiteQ[s1_]), kSiteQ[s2_]));
        if (be < 0) continue;
        for (int j = 0; j < SB.n[be]; ++j)
          cinfo.push_back(make_int4((s1_ * 4 + s2_) * rrp + SB.off[be] + j, s1_ * 4 + s2_, be, j));
      }
    A_.M = (int)rinfo.size() - A_.row0;
    A_.N = (int)cinfo.size() - A_.col0;
    p.flops1 += 2.0 * A_.M * (double)A_.N * A_.K;
    p.bytes1 += (double)A_.M * A_.K + (double)A_.K * A_.N + (double)A_.M * A_.N;
    for (int m0 = 0; m0 < A_.M; m0 += TILE)
      for (int c0 = 0; c0 < A_.N; c0 += TILE) tiles1.push_back(make_int4(a, m0, c0, 0));
  }
  p.ntiles1 = (int)tiles1.size();

  // stage 4 tables: charge classes of the output channels; in the panel of right
  // sector beta' the K index runs over the source sectors beta, and within one
  // over the channels of the class beta' - beta in channel order (rank), then j
  std::map<Q2, int> dcls;
  std::vector<int> ccls(RCx), crank(RCx);
  std::vector<std::vector<int>> members;
  for (int C = 0; C < RCx; ++C) {
    auto it = dcls.find(dC[C]);
    if (it == dcls.end()) {
      it = dcls.emplace(dC[C], (int)dcls.size()).first;
      members.emplace_back();
    }
    ccls[C] = it->second;
    crank[C] = (int)members[it->second].size();
    members[it->second].push_back(C);
  }
  p.ndcls = (int)dcls.size();
  std::vector<int> bshift((size_t)p.ndcls * nbe, -1);
  for (auto& kv : dcls)
    for (int be = 0; be < nbe; ++be) bshift[(size_t)kv.second * nbe + be] = SB.find(add(SB.q[be], kv.first));
  std::vector<int> kstart((size_t)nbe * nbe, -1), kbeta(nbe, 0);
  std::vector<BsPair> pairs;
  std::vector<long long> rbase(nbe, 0);
  long long nrs = 0;
  for (int bp = 0; bp < (p.wr ? 0 : nbe); ++bp) {
    rbase[bp] = nrs;
    for (int be = 0; be < nbe; ++be) {
      auto it = dcls.find(sub(SB.q[bp], SB.q[be]));
      if (it == dcls.end()) continue;
      kstart[(size_t)bp * nbe + be] = kbeta[bp];
      for (int C : members[it->second]) {
        pairs.push_back(BsPair{C, be, kbeta[bp], bp});
        kbeta[bp] += SB.n[be];
      }
    }
    nrs += (long long)kbeta[bp] * SB.n[bp];
  }
  p.nrs = nrs;
  p.npairs = (int)pairs.size();
  std::vector<long long> pbase((size_t)nal * 16 * nbe, -1), rowdst;
  std::vector<BsS4Tile> tiles4;
  std::vector<BsRedTile> red;
  long long n3 = 0;
  int slots = 0;
  p.flops4 = 0.0;
  p.bytes4 = 0.0;
  p.el_red = 0.0;
  for (int bp = 0; bp < (p.wr ? 0 : nbe); ++bp) {
    const int row0 = (int)rowdst.size();
    int M = 0;
    for (int a = 0; a < nal; ++a)
      for (int s1_ = 0; s1_ < 4; ++s1_)
        for (int s2_ = 0; s2_ < 4; ++s2_) {
          if (add(add(SA.q[a], kSiteQ[s1_]), kSiteQ[s2_]) != SB.q[bp]) continue;
          pbase[(((size_t)a * 4 + s1_) * 4 + s2_) * nbe + bp] = n3 + (long long)M * kbeta[bp];
          for (int i = 0; i < SA.n[a]; ++i)
            rowdst.push_back((long long)(SA.off[a] + i) * 16 * rrp + (long long)(s1_ * 4 + s2_) * rrp + SB.off[bp]);
          M += SA.n[a];
        }
    const int K = kbeta[bp], N = SB.n[bp];
    if (M > 0 && K > 0) {
      p.flops4 += 2.0 * M * (double)K * N;
      p.bytes4 += (double)M * K + (double)K * N + (double)M * N;
      for (int m0 = 0; m0 < M; m0 += TILE)
        for (int n0 = 0; n0 < N; n0 += TILE) {
          BsRedTile r{M, N, m0, n0, slots, 0, row0, 0};
          for (int k0 = 0; k0 < K; k0 += KSPLIT) {
            tiles4.push_back(BsS4Tile{n3, rbase[bp], M, N, K, m0, n0, k0, std::min(K, k0 + KSPLIT), slots});
            ++slots;
            ++r.nsplit;
          }
          p.el_red += (double)(r.nsplit + 1) * std::min(TILE, M - m0) * std::min(TILE, N - n0);
          red.push_back(r);
        }
    }
    n3 += (long long)M * K;
  }
  p.n3 = n3;
  if (p.wr) {
    tiles4.clear();
    red.swap(wred);
    rowdst.swap(wrowdst);
    slots = wslots;
    p.flops4 = wflops;
    p.bytes4 = wbytes;
    p.el_red = wel_red;
  }
  p.ntiles4 = p.wr ? p.nptiles : (int)tiles4.size();
  p.nred = (int)red.size();
  p.nslots = slots;

  hipStream_t s = E.stream;
  up(p.tiles1, tiles1, s);
  up(p.alpha, alpha, s);
  up(p.rsrc, rsrc, s);
  up(p.rinfo, rinfo, s);
  up(p.cinfo, cinfo, s);
  up(p.rowpart1, rowpart1, s);
  up(p.specoff, specoff, s);
  up(p.nbeta, SB.n, s);
  up(p.boff, SB.off, s);
  up(p.bshift, bshift, s);
  up(p.pbase, pbase, s);
  up(p.kbeta, kbeta, s);
  up(p.kstart, kstart, s);
  up(p.tiles4, tiles4, s);
  up(p.red, red, s);
  up(p.rowdst, rowdst, s);
  up(p.pairs, pairs, s);
  up(p.rbase, rbase, s);
  // mixes: site k (inputs T1 rows, outputs into T2) and site k+1 (inputs T2 rows, outputs into panels)
  // charge class of the second-mix output channels per group and output site state
  std::vector<std::array<int, 4>> gcls(ng);
  for (int g = 0; g < ng; ++g)
    for (int z = 0; z < 4; ++z) {
      auto it = dcls.find(sub(kSiteQ[z], gq[g]));
      gcls[g][z] = it == dcls.end() ? -1 : it->second;
    }
  std::vector<std::array<int, 4>> nocls(ng, std::array<int, 4>{-1, -1, -1, -1});
  if (!p.lw) {
    build_mix(E, p.m1, 1, w1, dB, RB, idx1, grp1, gid, gq, cols, ldg, off1, nr1, ns1, spec0, nspec, rowbase2, crank,
              nocls);
  } else {
    BsMix& m = p.m1;
    m.ntiles = m.nhtiles = m.nstage = m.noloc = m.nstaged = 0;
    m.flops = m.nin = m.nout = m.fl_light = m.el_light = m.fl_heavy = m.el_heavy = m.el_scatter = 0.0;
    m.ntmp = 0;
    m.heavy.clear();
  }
  if (!p.wr) {
    build_mix(E, p.m2, 2, w2, dC, RCx, idx2, grp2, gid, gq, cols, ldg, off2, nr2, ns2, spec0, nspec, rowbase2, crank,
              gcls);
  } else {
    BsMix& m = p.m2;
    m.ntiles = m.nhtiles = m.nstage = m.noloc = m.nstaged = 0;
    m.flops = m.nin = m.nout = m.fl_light = m.el_light = m.fl_heavy = m.el_heavy = m.el_scatter = 0.0;
    m.ntmp = 0;
    m.heavy.clear();
  }
  up(p.m1.spec, spec, s);
  up(p.m2.spec, spec, s);
  if (E.verbose_level >= 2) {
    std::fprintf(stderr, "[tt] window %d: rl %d rr %d groups %d stage-1 tiles %d stage-4 tiles %d; mix tiles %d/%d", b,
                 rlp, rrp, ng, p.ntiles1, p.ntiles4, p.m1.ntiles, p.m2.ntiles);
    for (int mi = 0; mi < 2; ++mi) {
      const BsMix& m = mi == 0 ? p.m1 : p.m2;
      std::fprintf(stderr, "; heavy GEMMs of mix %d (H x cols x Nin):", mi + 1);
      for (const BsHeavy& h : m.heavy) std::fprintf(stderr, " %dx%dx%d", h.H, h.cols, h.Nin);
    }
    if (p.lw)
      std::fprintf(stderr, "; left operator: %d groups, %d tiles, %lld elements, %.3g multiply-adds to form",
                   p.nlw_groups, p.nlw_tiles, p.nlw, p.build_lw);
    if (p.wr)
      std::fprintf(stderr, "; right operator: %d panels, %d chunks, %lld elements, %.3g multiply-adds to form",
                   p.npanels, p.nwr_items, p.nwr, p.build_wr);
    std::fprintf(stderr, "\n");
  }
  p.have64 = p.have32 = false;
  // unique over all engines: a workspace is zeroed again whenever it meets a plan it has not seen
  static std::atomic<long long> plan_serial{0};
  p.serial = ++plan_serial;
  p.ok = true;
  return true;
}

template <typename T>
static const DevMem& mix_vals(const BsMix& m);
template <>
const DevMem& mix_vals<double>(const BsMix& m) { return m.oval64; }
template <>
const DevMem& mix_vals<float>(const BsMix& m) { return m.oval32; }

template <typename T>
static const DevMem& heavy_vals(const BsMix& m);
template <>
const DevMem& heavy_vals<double>(const BsMix& m) { return m.hw64; }
template <>
const DevMem& heavy_vals<float>(const BsMix& m) { return m.hw32; }

// light rows gathered, heavy rows through the GEMM and a scatter pass
// descriptors of the heavy-row GEMMs of one mix (staging buffer E.bs_tmp, sized beforehand)
template <typename T>
static std::vector<GemmGroup<T>> heavy_groups(Engine& E, const BsMix& m, const T* in, long long nin) {
  std::vector<GemmGroup<T>> gg;
  const T* W = heavy_vals<T>(m).template as<T>();
  T* tmp = E.bs_tmp.as<T>();
  for (const BsHeavy& h : m.heavy) {
    if (h.in_base < 0 || h.in_base + (long long)h.Nin * h.ld > nin)
      throw std::runtime_error("block-sparse product: heavy rows read outside their group");
    GemmGroup<T> G{};
    G.g.M = h.H; G.g.N = h.cols; G.g.K = h.Nin; G.g.batch = 1; G.g.kin = ((h.Nin + 15) / 16) * 16;
    G.g.sAm = h.Nin4; G.g.sAkk = 1;
    G.g.sBkk = h.ld; G.g.sBn = 1;
    G.g.sCm = h.ld; G.g.alpha = 1.0; G.g.beta = 0.0;
    G.A = W + h.w_off;
    G.B = in + h.in_base;
    G.C = tmp + h.tmp_off;
    gg.push_back(G);
  }
  return gg;
}

// The heavy-row GEMMs of one mix split by their row count: buckets 0..2 run on the
// skinny streaming kernel (at most 16, 32, 64 rows), bucket 3 on the matrix-core tiles.
template <typename T>
static std::array<std::vector<GemmGroup<T>>, 4> split_heavy(const std::vector<GemmGroup<T>>& gg) {
  std::array<std::vector<GemmGroup<T>>, 4> parts;
  for (const GemmGroup<T>& G : gg) {
    const int mr = skinny_rows(G.g.M);
    parts[mr == 16 ? 0 : mr == 32 ? 1 : mr == 64 ? 2 : 3].push_back(G);
  }
  return parts;
}

template <typename T, int MODE>
static void run_mix(Engine& E, const BsPlan& p, const BsMix& m, const T* in, long long nin, T* out, long long nout,
                    int* err, bool rnd, const std::array<std::vector<GemmGroup<T>>, 4>& gg, DevMem* gdev) {
  hipStream_t s = E.stream;
  const int slot0 = MODE == 1 ? 1 : 4;
  if (m.ntiles > 0) {
    const size_t lds = m.nstaged > 0 ? sizeof(T) * MIX_STAGE * MIX_COLS : 0;
    hipLaunchKernelGGL((mix_kernel<T, MODE, false>), dim3(m.ntiles), dim3(MIX_COLS), lds, s, m.tiles.as<MixTile>(),
                       m.groups.as<BsGroup>(), m.rows.as<MixRow>(), m.ocol.as<int>(), mix_vals<T>(m).template as<T>(),
                       m.spec.as<int4>(), in, nin, out, nout, err, p.nbe, p.specoff.as<long long>(),
                       p.bshift.as<int>(), p.pbase.as<long long>(), p.kbeta.as<int>(), p.kstart.as<int>(),
                       p.nbeta.as<int>(), rnd ? 1 : 0, (const T*)nullptr, 0LL, m.stage.as<int>(), m.nstage, m.oloc.as<int>(), m.noloc);
    BSCHECK(hipGetLastError());
    E.kt_mark(slot0);
  }
  if (m.nhtiles > 0) {
    T* tmp = E.bs_tmp.as<T>();
    static const int kRows[3] = {16, 32, 64};
    for (int b = 0; b < 3; ++b)
      if (!gg[b].empty()) gemm_grouped_skinny<T>(gdev[b].template as<GemmGroup<T>>(), gg[b], kRows[b], s);
    if (!gg[3].empty()) gemm_grouped<T>(gdev[3].template as<GemmGroup<T>>(), gg[3], s);
    E.kt_mark(slot0 + 1);
    hipLaunchKernelGGL((mix_kernel<T, MODE, true>), dim3(m.nhtiles), dim3(MIX_COLS), 0, s, m.htiles.as<MixTile>(),
                       m.groups.as<BsGroup>(), m.hrows.as<MixRow>(), m.ocol.as<int>(), mix_vals<T>(m).template as<T>(),
                       m.spec.as<int4>(), in, nin, out, nout, err, p.nbe, p.specoff.as<long long>(),
                       p.bshift.as<int>(), p.pbase.as<long long>(), p.kbeta.as<int>(), p.kstart.as<int>(),
                       p.nbeta.as<int>(), rnd ? 1 : 0, (const T*)tmp, m.ntmp, m.stage.as<int>(), m.nstage, m.oloc.as<int>(), m.noloc);
    BSCHECK(hipGetLastError());
    E.kt_mark(slot0 + 2);
  }
}

template <typename T>
void bs_apply(Engine& E, BsPlan& p, const T* L, const T* R, const T* Rt, const T* x, T* y, bool bf16_t3,
              bool check) {
  if (!p.ok) throw std::runtime_error("block-sparse plan not built");
  hipStream_t s = E.stream;
  // bfloat16 with both operators precontracted: LW, WR, x and the chunk stores are held in
  // bfloat16 (FP32 arithmetic); otherwise every operand has the type T
  const bool b16 = sizeof(T) == 4 && bf16_t3 && p.wr;
  const int prec = sizeof(T) == 8 ? 0 : (b16 ? 2 : 1);
  const size_t es2 = b16 ? sizeof(uint16_t) : sizeof(T);  // element of the chunk stores / T2
  const size_t ny = (size_t)p.rlp * 16 * p.rrp;
  if (!p.err.p) p.err.resize_zero(sizeof(int), s);
  int* err = p.err.as<int>();
  if (!p.lw) E.bs_t1.ensure(sizeof(T) * std::max<long long>(p.n1, 1));
  E.bs_t2.ensure(es2 * std::max<long long>(p.n2, 1));
  E.bs_t3.ensure(sizeof(T) * std::max<long long>(p.n3, 1));
  E.bs_part.ensure(sizeof(T) * (size_t)std::max(p.nslots, 1) * TILE * TILE);
  if (E.bs_zero_serial != p.serial || E.bs_zero_prec != prec) {
    // entries that are never written: T1's where the left sector alpha' - d_A does not
    // exist; with the left operator T2's of the rows (B, s1') without operator entries
    if (p.lw) fill(E.bs_t2.p, es2 * p.n2, s);
    else fill(E.bs_t1.p, sizeof(T) * p.n1, s);
    E.bs_zero_serial = p.serial;
    E.bs_zero_prec = prec;
  }
  const T* lwop = nullptr;
  auto bf16_copy = [&](const DevMem& from, DevMem& to, long long n, bool& have) {
    if (have) return;
    to.ensure(sizeof(uint16_t) * (size_t)std::max<long long>(n, 1));
    if (n > 0) {
      const int nb = (int)std::min<long long>((n + 255) / 256, 8192);
      hipLaunchKernelGGL((to_bf16_kernel<double>), dim3(nb), dim3(256), 0, s, from.as<double>(), to.as<uint16_t>(), n);
      BSCHECK(hipGetLastError());
    }
    have = true;
  };
  if (b16) {
    if (!p.have_lw64) throw std::logic_error("block-sparse product: left operator not formed");
    bf16_copy(p.lw64, p.lw16, p.nlw, p.have_lw16);
    bf16_copy(p.wr64, p.wr16, p.nwr, p.have_wr16);
    E.bs_x16.ensure(sizeof(uint16_t) * ny);
    const int nb = (int)std::min<long long>(((long long)ny + 255) / 256, 8192);
    hipLaunchKernelGGL((to_bf16_kernel<T>), dim3(nb), dim3(256), 0, s, x, E.bs_x16.as<uint16_t>(), (long long)ny);
    BSCHECK(hipGetLastError());
  } else if (p.lw) {
    if (!p.have_lw64) throw std::logic_error("block-sparse product: left operator not formed");
    if (sizeof(T) == 8) {
      lwop = reinterpret_cast<const T*>(p.lw64.p);
    } else {
      const int want = bf16_t3 ? 2 : 1;
      if (p.lw32_state != want) {
        p.lw32.ensure(sizeof(float) * (size_t)std::max<long long>(p.nlw, 1));
        if (p.nlw > 0) {
          const int nb = (int)std::min<long long>((p.nlw + 255) / 256, 8192);
          hipLaunchKernelGGL(operator_f32_kernel, dim3(nb), dim3(256), 0, s, p.lw64.as<double>(), p.lw32.as<float>(),
                             p.nlw, want == 2 ? 1 : 0);
          BSCHECK(hipGetLastError());
        }
        p.lw32_state = want;
      }
      lwop = reinterpret_cast<const T*>(p.lw32.p);
    }
  }
  DevMem& rs = prec == 0 ? p.rstack64 : p.rstack32;
  bool& have = prec == 0 ? p.have64 : p.have32;
  if (!have) {
    rs.ensure(sizeof(T) * std::max<long long>(p.nrs, 1));
    if (p.npairs > 0) {
      if (p.RCx > p.RC && !Rt) throw std::runtime_error("block-sparse product: missing block environment");
      hipLaunchKernelGGL((rstack_kernel<T>), dim3(p.npairs), dim3(256), 0, s, p.pairs.as<BsPair>(), p.boff.as<int>(),
                         p.nbeta.as<int>(), p.rbase.as<long long>(), p.RC, p.RCx, p.rrp, R, Rt, rs.as<T>(), p.nrs,
                         err);
      BSCHECK(hipGetLastError());
    }
    have = true;
  }
  fill(y, sizeof(T) * ny, s);
  // heavy-row GEMM descriptors uploaded before the timed kernels
  E.bs_tmp.ensure(sizeof(T) * std::max<long long>(std::max(p.m1.ntmp, p.m2.ntmp), 1));
  const auto gg1 = split_heavy<T>(heavy_groups<T>(E, p.m1, E.bs_t1.as<T>(), p.n1));
  const auto gg2 = split_heavy<T>(heavy_groups<T>(E, p.m2, E.bs_t2.as<T>(), p.n2));
  // the descriptors change only with the plan, the precision or the workspace addresses
  if (E.bs_gg_serial != p.serial || E.bs_gg_prec != prec || E.bs_gg_ptr[0] != E.bs_t1.p ||
      E.bs_gg_ptr[1] != E.bs_t2.p || E.bs_gg_ptr[2] != E.bs_tmp.p) {
    for (int b = 0; b < 4; ++b) {
      if (!gg1[b].empty()) upload(E.bs_gg1[b], gg1[b].data(), gg1[b].size() * sizeof(GemmGroup<T>), s);
      if (!gg2[b].empty()) upload(E.bs_gg2[b], gg2[b].data(), gg2[b].size() * sizeof(GemmGroup<T>), s);
    }
    E.bs_gg_serial = p.serial;
    E.bs_gg_prec = prec;
    E.bs_gg_ptr[0] = E.bs_t1.p;
    E.bs_gg_ptr[1] = E.bs_t2.p;
    E.bs_gg_ptr[2] = E.bs_tmp.p;
  }
  const T* wrop = nullptr;
  if (p.wr && !b16) {
    if (sizeof(T) == 8) {
      wrop = reinterpret_cast<const T*>(p.wr64.p);
    } else {
      const int want = bf16_t3 ? 2 : 1;
      if (p.wr32_state != want) {
        p.wr32.ensure(sizeof(float) * (size_t)std::max<long long>(p.nwr, 1));
        if (p.nwr > 0) {
          const int nb = (int)std::min<long long>((p.nwr + 255) / 256, 8192);
          hipLaunchKernelGGL(operator_f32_kernel, dim3(nb), dim3(256), 0, s, p.wr64.as<double>(), p.wr32.as<float>(),
                             p.nwr, want == 2 ? 1 : 0);
          BSCHECK(hipGetLastError());
        }
        p.wr32_state = want;
      }
      wrop = reinterpret_cast<const T*>(p.wr32.p);
    }
  }
  E.kt_begin();
  if (p.lw) {
    if (p.nlw_tiles > 0) {
      if (b16) {
        if constexpr (sizeof(T) == 4)
          hipLaunchKernelGGL((lw_gemm_kernel<float, 2, uint16_t>), dim3(p.nlw_tiles), dim3(256), 0, s,
                             p.lw_tiles.as<BsLwTile>(), p.lw_groups.as<BsLwGroup>(), p.lw_blocks.as<BsLwBlock>(),
                             p.lw_krow.as<int>(), p.lw_col.as<int2>(), p.lw16.as<uint16_t>(), p.nlw,
                             E.bs_x16.as<uint16_t>(), (long long)ny, (const long long*)nullptr,
                             (const long long*)nullptr, p.nbeta.as<int>(), p.nbe, p.lw_zeta.as<BsZeta>(),
                             p.lw_kc.as<int>(), E.bs_t2.as<uint16_t>(), p.n2, err);
      } else if (p.wr) {
        hipLaunchKernelGGL((lw_gemm_kernel<T, 2, T>), dim3(p.nlw_tiles), dim3(256), 0, s, p.lw_tiles.as<BsLwTile>(),
                           p.lw_groups.as<BsLwGroup>(), p.lw_blocks.as<BsLwBlock>(),
                           p.lw_krow.as<int>(), p.lw_col.as<int2>(), lwop, p.nlw, x, (long long)ny, (const long long*)nullptr,
                           (const long long*)nullptr, p.nbeta.as<int>(), p.nbe, p.lw_zeta.as<BsZeta>(),
                           p.lw_kc.as<int>(), E.bs_t2.as<T>(), p.n2, err);
      } else {
        hipLaunchKernelGGL((lw_gemm_kernel<T, 1, T>), dim3(p.nlw_tiles), dim3(256), 0, s, p.lw_tiles.as<BsLwTile>(),
                           p.lw_groups.as<BsLwGroup>(), p.lw_blocks.as<BsLwBlock>(),
                           p.lw_krow.as<int>(), p.lw_col.as<int2>(), lwop, p.nlw, x, (long long)ny, p.rowbase2.as<long long>(),
                           p.specoff.as<long long>(), p.nbeta.as<int>(), p.nbe, (const BsZeta*)nullptr,
                           (const int*)nullptr, E.bs_t2.as<T>(), p.n2, err);
      }
      BSCHECK(hipGetLastError());
      E.kt_mark(0);
    }
  } else {
    if (p.ntiles1 > 0) {
      hipLaunchKernelGGL((stage1_mfma_kernel<T>), dim3(p.ntiles1), dim3(256), 0, s, p.tiles1.as<int4>(),
                         p.alpha.as<BsAlpha>(), p.rsrc.as<long long>(), p.rinfo.as<int4>(), p.cinfo.as<int4>(),
                         p.rowpart1.as<long long>(), p.specoff.as<long long>(), p.nbeta.as<int>(), p.nbe, L,
                         (long long)p.RAx * p.rlp * p.rlp, x, (long long)ny, (long long)16 * p.rrp, E.bs_t1.as<T>(),
                         p.n1, err);
      BSCHECK(hipGetLastError());
    }
    if (p.ntiles1 > 0) E.kt_mark(0);
    run_mix<T, 1>(E, p, p.m1, E.bs_t1.as<T>(), p.n1, E.bs_t2.as<T>(), p.n2, err, false, gg1, E.bs_gg1);
  }
  if (!p.wr) run_mix<T, 2>(E, p, p.m2, E.bs_t2.as<T>(), p.n2, E.bs_t3.as<T>(), p.n3, err, bf16_t3, gg2, E.bs_gg2);
  if (p.ntiles4 > 0) {
    // panels x WR (right operator), or stage-4 panels x stacked R
    if (b16) {
      if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((panel_mfma_kernel<float, uint16_t>), dim3(p.ntiles4), dim3(256), 0, s,
                           p.wr_ptiles.as<BsPTile>(), p.wr_k8.as<BsK8>(), p.nk8, E.bs_t2.as<uint16_t>(), p.n2,
                           p.wr16.as<uint16_t>(), p.nwr, E.bs_part.as<float>(), err);
    } else if (p.wr)
      hipLaunchKernelGGL((panel_mfma_kernel<T, T>), dim3(p.ntiles4), dim3(256), 0, s, p.wr_ptiles.as<BsPTile>(),
                         p.wr_k8.as<BsK8>(), p.nk8, E.bs_t2.as<T>(), p.n2, wrop, p.nwr, E.bs_part.as<T>(), err);
    else
      hipLaunchKernelGGL((stage4_mfma_kernel<T>), dim3(p.ntiles4), dim3(256), 0, s, p.tiles4.as<BsS4Tile>(),
                         E.bs_t3.as<T>(), p.n3, rs.as<T>(), p.nrs, E.bs_part.as<T>(), err);
    BSCHECK(hipGetLastError());
    E.kt_mark(7);
    hipLaunchKernelGGL((reduce4_kernel<T>), dim3(p.nred), dim3(256), 0, s, p.red.as<BsRedTile>(),
                       E.bs_part.as<T>(), p.rowdst.as<long long>(), y, (long long)ny, err);
    BSCHECK(hipGetLastError());
    E.kt_mark(8);
  }
  if (check) bs_check(E, p);
  const double el = (double)sizeof(T), elw = b16 ? (double)sizeof(uint16_t) : el;
  const double fl[Engine::KT_SLOTS] = {p.lw ? p.flops_lw : p.flops1, p.m1.fl_light, p.m1.fl_heavy, 0.0,
                                       p.m2.fl_light, p.m2.fl_heavy, 0.0, p.flops4, 0.0};
  const double by[Engine::KT_SLOTS] = {elw * (p.lw ? p.bytes_lw : p.bytes1), el * p.m1.el_light, el * p.m1.el_heavy,
                                       el * p.m1.el_scatter,
                                       el * p.m2.el_light, el * p.m2.el_heavy, el * p.m2.el_scatter, elw * p.bytes4,
                                       el * p.el_red};
  E.kt_end(fl, by);
}

// split-K panel x stacked-matrix products of the one-site product (same kernels as stage 4)
void bs_splitk_tables(const std::vector<BsSplitSeg>& segs, std::vector<BsS4Tile>& tiles, std::vector<BsRedTile>& red,
                      int& nslots, double& el_red) {
  tiles.clear();
  red.clear();
  nslots = 0;
  el_red = 0.0;
  for (const BsSplitSeg& g : segs) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) continue;
    for (int m0 = 0; m0 < g.M; m0 += TILE)
      for (int n0 = 0; n0 < g.N; n0 += TILE) {
        BsRedTile r{g.M, g.N, m0, n0, nslots, 0, g.row0, 0};
        for (int k0 = 0; k0 < g.K; k0 += KSPLIT) {
          tiles.push_back(BsS4Tile{g.abase, g.bbase, g.M, g.N, g.K, m0, n0, k0, std::min(g.K, k0 + KSPLIT), nslots});
          ++nslots;
          ++r.nsplit;
        }
        el_red += (double)(r.nsplit + 1) * std::min(TILE, g.M - m0) * std::min(TILE, g.N - n0);
        red.push_back(r);
      }
  }
}

void bs_splitk_run(Engine& E, int ntiles, const BsS4Tile* tiles, int nred, const BsRedTile* red,
                   const long long* rowdst, const double* A, long long nA, const double* B, long long nB, double* part,
                   double* y, long long ny, int* err, int slot_gemm, int slot_red) {
  hipStream_t s = E.stream;
  if (ntiles <= 0) return;
  hipLaunchKernelGGL((stage4_mfma_kernel<double>), dim3(ntiles), dim3(256), 0, s, tiles, A, nA, B, nB, part, err);
  BSCHECK(hipGetLastError());
  if (slot_gemm >= 0) E.kt_mark(slot_gemm);
  hipLaunchKernelGGL((reduce4_kernel<double>), dim3(nred), dim3(256), 0, s, red, part, rowdst, y, ny, err);
  BSCHECK(hipGetLastError());
  if (slot_red >= 0) E.kt_mark(slot_red);
}

void bs_lw_build(Engine& E, BsPlan& p, const double* L, long long nL, const double* R, const double* Rt) {
  if (!p.ok || !p.lw) throw std::logic_error("bs_lw_build: plan without a left operator");
  if (p.wr && (!R || (p.RCx > p.RC && !Rt))) throw std::logic_error("bs_lw_build: missing right environment");
  hipStream_t s = E.stream;
  if (!p.err.p) p.err.resize_zero(sizeof(int), s);
  p.lw64.ensure(sizeof(double) * (size_t)std::max<long long>(p.nlw, 1));
  if (p.nlw_blocks > 0) {
    hipLaunchKernelGGL(lw_build_kernel, dim3(p.nlw_blocks), dim3(256), 0, s, p.lw_blocks.as<BsLwBlock>(),
                       p.lw_groups.as<BsLwGroup>(), p.lw_tptr.as<int>(), p.lw_tA.as<int>(), p.lw_tv.as<double>(),
                       p.aoff.as<int>(), L, nL, p.rlp, p.lw64.as<double>(), p.nlw, p.err.as<int>());
    BSCHECK(hipGetLastError());
  }
  if (p.wr) {
    p.wr64.ensure(sizeof(double) * (size_t)std::max<long long>(p.nwr, 1));
    fill(p.wr64.p, sizeof(double) * (size_t)p.nwr, s);  // rows of the chunk padding stay zero
    if (p.nwr_items > 0) {
      const long long rr2 = (long long)p.rrp * p.rrp;
      hipLaunchKernelGGL(wr_build_kernel, dim3(p.nwr_items), dim3(256), 0, s, p.wr_items.as<BsWrItem>(),
                         p.wr_panels.as<BsPanel>(), p.wr_tptr.as<int>(), p.wr_tC.as<int>(), p.wr_tv.as<double>(),
                         p.boff.as<int>(), p.nbeta.as<int>(), R, (long long)p.RC * rr2, Rt,
                         (long long)(p.RCx - p.RC) * rr2, p.RC, p.rrp, p.wr64.as<double>(), p.nwr, p.err.as<int>());
      BSCHECK(hipGetLastError());
    }
  }
  p.have_lw64 = true;
  p.lw32_state = p.wr32_state = 0;
  p.have_lw16 = p.have_wr16 = false;
  bs_check(E, p);
}

void bs_check(Engine& E, BsPlan& p) {
  int herr = 0;
  BSCHECK(hipMemcpyAsync(&herr, p.err.as<int>(), sizeof(int), hipMemcpyDeviceToHost, E.stream));
  BSCHECK(hipStreamSynchronize(E.stream));
  if (herr != 0)
    throw std::runtime_error("block-sparse product: index outside its buffer (check " + std::to_string(herr) + ")");
}

template void bs_apply<double>(Engine&, BsPlan&, const double*, const double*, const double*, const double*, double*,
                               bool, bool);
template void bs_apply<float>(Engine&, BsPlan&, const float*, const float*, const float*, const float*, float*, bool,
                              bool);

}  // namespace tt
