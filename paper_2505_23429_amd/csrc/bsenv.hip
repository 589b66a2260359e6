// Quantum-number block-sparse environment update through one site (FP64).
// Layout and index conventions are described in bsheff.h.
//
// Bond roles: P = bra at the input bond, Q = ket at the input bond,
// R = ket at the output bond, T = bra at the output bond.  With sigma = +1
// (left update) the cores are read as ket[q][s][r], bra[p][s'][t]; with
// sigma = -1 (right update) as ket[r][s][q], bra[t][s'][p].
//   stage 1  T1[(K, s)][spec(pi, rho)] = sum_q E_K[p][q] ket(q, s, r)   grouped GEMM per (class, kappa)
//   mix      panel_tau[(pi, s', i_p)][(K', i_r)] = sum W T1                sparse x dense per group
//   stage 3  out[K'][t][r] = sum_k bra(p, s', t) panel_tau                 grouped GEMM per (tau, class)
#include "bsheff.h"

#include <algorithm>
#include <map>
#include <stdexcept>

namespace tt {

#define BECHECK(x)                                                                   \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) throw tt::HipError(std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

namespace {

const Q2 kQ[4] = {{0, 0}, {1, 1}, {1, -1}, {2, 0}};  // (N, 2Sz) of |0>, |up>, |dn>, |up dn>
inline Q2 add(Q2 a, Q2 b) { return {a[0] + b[0], a[1] + b[1]}; }
inline Q2 sub(Q2 a, Q2 b) { return {a[0] - b[0], a[1] - b[1]}; }
inline Q2 mul(int s, Q2 a) { return {s * a[0], s * a[1]}; }

constexpr int TL = 64;   // GEMM output tile edge
constexpr int KS = 32;   // K slice in LDS
constexpr int MC = 256;  // mix: spectator columns per workgroup
constexpr int MR = 64;   // mix: output rows per workgroup
constexpr int HEAVY = 32;  // output rows with more operator entries go through the dense GEMM

struct Sec {
  std::vector<Q2> q;
  std::vector<int> off, n;
  std::map<Q2, int> id;
  int find(Q2 c) const {
    auto it = id.find(c);
    return it == id.end() ? -1 : it->second;
  }
};

bool sectors(const Labels& lab, Sec& s) {
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

template <class V>
void up(DevMem& d, const std::vector<V>& v, hipStream_t s) {
  if (v.empty()) {
    const V z{};
    upload(d, &z, sizeof(V), s);
  } else {
    upload(d, v.data(), v.size() * sizeof(V), s);
  }
}

struct EnvS1 { int M, N, K, cls0, np, op, oq, col0, pi, pad; };
struct EnvGrp { long long in_base; int ncols, spec0, nspec, ld; };  // ld: row stride of T1 (multiple of 4)
struct EnvS3 { long long upoff, pbase; int M, N, K, ld, pcol, cls0, nrho, orho, otau, pad; };
struct EnvUP { long long upoff; int tau, pi, s, koff, K, pad; };

// stage 1: rows (K in the input class, i_p), columns (s, rho, i_r), sum over the ket sector kappa
__global__ __launch_bounds__(256) void env_s1_kernel(
    const int4* __restrict__ tiles, const EnvS1* __restrict__ desc, const int* __restrict__ clist_in,
    const int4* __restrict__ cinfo, const int* __restrict__ gidx, const int* __restrict__ rin,
    const long long* __restrict__ goff, const int* __restrict__ gcols, const long long* __restrict__ specoff,
    const int* __restrict__ nR, int nRsec, const double* __restrict__ Ein, long long PQ, int Qp, long long nE,
    const double* __restrict__ ket, long long nket, long long bks, double* __restrict__ T1, long long n1,
    int* __restrict__ err) {
  const int4 t = tiles[blockIdx.x];
  const EnvS1 d = desc[t.x];
  const int m0 = t.y, c0 = t.z;
  __shared__ double As[KS][TL + 1];
  __shared__ double Bs[KS][TL + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < d.K; k0 += KS) {
    for (int e = tid; e < TL * KS; e += 256) {
      const int r = e / KS, kk = e % KS;
      double v = 0.0;
      if (m0 + r < d.M && k0 + kk < d.K) {
        const int m = m0 + r;
        const int K = clist_in[d.cls0 + m / d.np];
        const long long q = (long long)K * PQ + (long long)(d.op + m % d.np) * Qp + d.oq + k0 + kk;
        if (q >= 0 && q < nE) v = Ein[q]; else err[0] = 11;
      }
      As[kk][r] = v;
    }
    for (int e = tid; e < TL * KS; e += 256) {
      const int kk = e / TL, c = e % TL;
      double v = 0.0;
      if (c0 + c < d.N && k0 + kk < d.K) {
        const long long q = (long long)(d.oq + k0 + kk) * bks + cinfo[d.col0 + c0 + c].x;
        if (q >= 0 && q < nket) v = ket[q]; else err[0] = 12;
      }
      Bs[kk][c] = v;
    }
    __syncthreads();
    const int kn = min(KS, d.K - k0);
    for (int kk = 0; kk < kn; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= d.M) continue;
    const int K = clist_in[d.cls0 + m / d.np], ip = m % d.np;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tx + 16 * j;
      if (c >= d.N) continue;
      const int4 ci = cinfo[d.col0 + c];  // {ket column, s, rho, i_r}
      const int g = gidx[K * 4 + ci.y];
      const long long so = specoff[(long long)d.pi * nRsec + ci.z];
      if (g < 0 || so < 0) { err[0] = 13; continue; }
      const long long dst = goff[g] + (long long)rin[K * 4 + ci.y] * gcols[g] + so + (long long)ip * nR[ci.z] + ci.w;
      if (dst < 0 || dst >= n1) { err[0] = 14; continue; }
      T1[dst] = acc[i][j];
    }
  }
}

// mix: output row (K', s') of a group, one spectator column per thread, written into the panel of tau
__global__ __launch_bounds__(MC) void env_mix_kernel(
    const int4* __restrict__ tiles, const EnvGrp* __restrict__ grp, const int* __restrict__ optr,
    const int* __restrict__ ocol, const double* __restrict__ oval, const int2* __restrict__ orow,
    const int4* __restrict__ spec, const double* __restrict__ T1, long long n1, double* __restrict__ panel,
    long long npan, const int* __restrict__ t3tau, const long long* __restrict__ t3base, const int* __restrict__ Ntau,
    const int* __restrict__ pcol, int ncout, const int* __restrict__ cls_out, const int* __restrict__ pos_out,
    const int* __restrict__ nR, int* __restrict__ err, const long long* __restrict__ hbase,
    const double* __restrict__ tmp) {
  const int4 t = tiles[blockIdx.x];
  const EnvGrp G = grp[t.x];
  const int col = t.y + (int)threadIdx.x;
  if (col >= G.ncols) return;
  int lo = 0, hi = G.nspec - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (spec[G.spec0 + mid].x <= col) lo = mid; else hi = mid - 1;
  }
  const int4 sp = spec[G.spec0 + lo];  // {start, pi, rho, -}
  const int within = col - sp.x;
  const int nr = nR[sp.z];
  const int ip = within / nr, ir = within - ip * nr;
  const long long lim = n1 - G.in_base - col;
  const double* src = T1 + G.in_base + col;
  for (int r = t.z; r < t.w; ++r) {
    double acc = 0.0;
    if (hbase) {
      acc = tmp[hbase[r] + col];  // heavy row: sum formed by the GEMM
    } else {
      const int e1 = optr[r + 1];
      for (int e = optr[r]; e < e1; ++e) {
        const long long q = (long long)ocol[e] * G.ld;
        if (q >= 0 && q < lim) acc += oval[e] * src[q]; else err[0] = 15;
      }
    }
    const int2 ro = orow[r];  // {K', s'}
    const int ts = sp.y * 4 + ro.y;
    const int tau = t3tau[ts];
    if (tau < 0) continue;
    const long long dst = t3base[ts] + (long long)ip * Ntau[tau] + pcol[tau * ncout + cls_out[ro.x]] +
                          (long long)pos_out[ro.x] * nr + ir;
    if (dst < 0 || dst >= npan) { err[0] = 16; continue; }
    panel[dst] = acc;
  }
}

// bra panel of tau: UP[m][koff + i_p] = bra(p = o_pi + i_p, s', t = o_tau + m)
__global__ __launch_bounds__(256) void env_up_kernel(const EnvUP* __restrict__ ups, const double* __restrict__ bra,
                                                     long long nbra, long long ps, long long ss, long long ts,
                                                     const int* __restrict__ oP, const int* __restrict__ nP,
                                                     const int* __restrict__ oT, const int* __restrict__ nT,
                                                     double* __restrict__ UP, long long nup, int* __restrict__ err) {
  const EnvUP u = ups[blockIdx.x];
  const int np = nP[u.pi], nt = nT[u.tau];
  for (int e = threadIdx.x; e < np * nt; e += 256) {
    const int m = e / np, ip = e - m * np;
    const long long q = (long long)(oP[u.pi] + ip) * ps + (long long)u.s * ss + (long long)(oT[u.tau] + m) * ts;
    const long long dst = u.upoff + (long long)m * u.K + u.koff + ip;
    if (q < 0 || q >= nbra || dst < 0 || dst >= nup) { err[0] = 17; continue; }
    UP[dst] = bra[q];
  }
}

// stage 3: out[K'][o_tau + m][o_rho + i_r] = sum_k UP[m][k] panel[k][pcol + (K' position, i_r)]
__global__ __launch_bounds__(256) void env_s3_kernel(const int4* __restrict__ tiles, const EnvS3* __restrict__ desc,
                                                     const double* __restrict__ UP, long long nup,
                                                     const double* __restrict__ panel, long long npan,
                                                     const int* __restrict__ clist_out, double* __restrict__ out,
                                                     long long nout, long long TR, int Rp, int* __restrict__ err) {
  const int4 t = tiles[blockIdx.x];
  const EnvS3 d = desc[t.x];
  const int m0 = t.y, n0 = t.z;
  __shared__ double As[KS][TL + 1];
  __shared__ double Bs[KS][TL + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < d.K; k0 += KS) {
    for (int e = tid; e < TL * KS; e += 256) {
      const int r = e / KS, kk = e % KS;
      double v = 0.0;
      if (m0 + r < d.M && k0 + kk < d.K) {
        const long long q = d.upoff + (long long)(m0 + r) * d.K + k0 + kk;
        if (q >= 0 && q < nup) v = UP[q]; else err[0] = 18;
      }
      As[kk][r] = v;
    }
    for (int e = tid; e < TL * KS; e += 256) {
      const int kk = e / TL, c = e % TL;
      double v = 0.0;
      if (n0 + c < d.N && k0 + kk < d.K) {
        const long long q = d.pbase + (long long)(k0 + kk) * d.ld + d.pcol + n0 + c;
        if (q >= 0 && q < npan) v = panel[q]; else err[0] = 19;
      }
      Bs[kk][c] = v;
    }
    __syncthreads();
    const int kn = min(KS, d.K - k0);
    for (int kk = 0; kk < kn; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= d.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx + 16 * j;
      if (n >= d.N) continue;
      const int K = clist_out[d.cls0 + n / d.nrho], ir = n % d.nrho;
      const long long dst = (long long)K * TR + (long long)(d.otau + m) * Rp + d.orho + ir;
      if (dst < 0 || dst >= nout) { err[0] = 20; continue; }
      out[dst] = acc[i][j];
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// site tables
// ---------------------------------------------------------------------------
void bs_site_use(Engine& E, BsSiteUse& u, const SiteOp& op, const std::vector<Q2>& din,
                 const std::vector<Q2>& dout, int sigma) {
  u = BsSiteUse();
  u.sigma = sigma;
  u.nin = (int)din.size();
  u.nout = (int)dout.size();
  if (op.nout != u.nout) throw std::runtime_error("block-sparse site tables: channel count mismatch");
  auto classes = [](const std::vector<Q2>& d, std::vector<Q2>& cq, std::vector<int>& cls, std::vector<int>& cstart,
                    std::vector<int>& clist, std::vector<int>& pos) {
    std::map<Q2, int> m;
    for (const Q2& q : d) m.emplace(q, 0);
    int c = 0;
    for (auto& kv : m) { kv.second = c++; cq.push_back(kv.first); }
    cls.resize(d.size());
    std::vector<int> cnt(c, 0);
    for (size_t k = 0; k < d.size(); ++k) { cls[k] = m[d[k]]; cnt[cls[k]]++; }
    cstart.assign(c + 1, 0);
    for (int i = 0; i < c; ++i) cstart[i + 1] = cstart[i] + cnt[i];
    clist.resize(d.size());
    pos.resize(d.size());
    std::vector<int> fill = cstart;
    for (size_t k = 0; k < d.size(); ++k) {
      pos[k] = fill[cls[k]] - cstart[cls[k]];
      clist[fill[cls[k]]++] = (int)k;
    }
    return c;
  };
  std::vector<int> clist_in, clist_out, pos_in, pos_out;
  u.ncin = classes(din, u.cq_in, u.cls_in, u.cstart_in, clist_in, pos_in);
  u.ncout = classes(dout, u.cq_out, u.cls_out, u.cstart_out, clist_out, pos_out);
  auto group = [&](Q2 G) {
    auto it = u.gid.find(G);
    if (it != u.gid.end()) return it->second;
    const int g = (int)u.gq.size();
    u.gid[G] = g;
    u.gq.push_back(G);
    return g;
  };
  std::vector<int> rin(u.nin * 4), nrows;
  u.gidx_in.assign(u.nin * 4, -1);
  for (int K = 0; K < u.nin; ++K)
    for (int s = 0; s < 4; ++s) {
      const int g = group(sub(mul(sigma, kQ[s]), din[K]));
      if ((int)nrows.size() <= g) nrows.resize(g + 1, 0);
      u.gidx_in[K * 4 + s] = g;
      rin[K * 4 + s] = nrows[g]++;
    }
  std::vector<std::vector<int2>> rows_by_g;
  for (int K = 0; K < u.nout; ++K)
    for (int s = 0; s < 4; ++s) {
      const int g = group(sub(mul(sigma, kQ[s]), dout[K]));
      if ((int)rows_by_g.size() <= g) rows_by_g.resize(g + 1);
      rows_by_g[g].push_back(make_int2(K, s));
    }
  u.ngrp = (int)u.gq.size();
  rows_by_g.resize(u.ngrp);
  nrows.resize(u.ngrp, 0);
  std::vector<int> optr(1, 0), ocol;
  std::vector<double> oval, hw;
  std::vector<int2> orow, hrow;
  u.orow0.assign(u.ngrp + 1, 0);
  u.hrow0.assign(u.ngrp + 1, 0);
  u.nin4.assign(u.ngrp, 0);
  u.hw_off.assign(u.ngrp, 0);
  u.nnz = 0.0;
  u.nent_light.assign(u.ngrp, 0.0);
  nrows.resize(u.ngrp, 0);
  std::vector<std::pair<int, double>> ent;
  for (int g = 0; g < u.ngrp; ++g) {
    u.orow0[g] = (int)orow.size();
    u.hrow0[g] = (int)hrow.size();
    u.nin4[g] = (nrows[g] + 3) / 4 * 4;
    u.hw_off[g] = (long long)hw.size();
    for (const int2& ro : rows_by_g[g]) {
      ent.clear();
      for (int e = op.hptr[ro.x]; e < op.hptr[ro.x + 1]; ++e) {
        const int Kin = op.hsrc[e];
        if (Kin < 0 || Kin >= u.nin) throw std::runtime_error("block-sparse site tables: input channel out of range");
        for (int s = 0; s < 4; ++s) {
          const double v = op.hop[(size_t)e * 16 + ro.y * 4 + s];
          if (v == 0.0) continue;
          if (u.gidx_in[Kin * 4 + s] != g)
            throw std::runtime_error("block-sparse site tables: operator entry breaks the charge grouping");
          ent.emplace_back(rin[Kin * 4 + s], v);
        }
      }
      u.nnz += (double)ent.size();
      if ((int)ent.size() > HEAVY) {
        const size_t base = hw.size();
        hw.resize(base + u.nin4[g], 0.0);
        for (auto& pv : ent) hw[base + pv.first] += pv.second;
        hrow.push_back(ro);
        continue;
      }
      for (auto& pv : ent) { ocol.push_back(pv.first); oval.push_back(pv.second); }
      u.nent_light[g] += (double)ent.size();
      optr.push_back((int)ocol.size());
      orow.push_back(ro);
    }
  }
  u.orow0[u.ngrp] = (int)orow.size();
  u.hrow0[u.ngrp] = (int)hrow.size();
  u.nrows_in = nrows;
  up(u.hrow, hrow, E.stream);
  up(u.hw, hw, E.stream);
  hipStream_t st = E.stream;
  up(u.clist_in, clist_in, st);
  up(u.clist_out, clist_out, st);
  up(u.pos_out, pos_out, st);
  up(u.d_cls_out, u.cls_out, st);
  up(u.d_gidx_in, u.gidx_in, st);
  up(u.rin, rin, st);
  up(u.optr, optr, st);
  up(u.ocol, ocol, st);
  up(u.oval, oval, st);
  up(u.orow, orow, st);
}

// ---------------------------------------------------------------------------
// tables of one update shape (bond labels and padded sizes), and the first two
// stages (stage 1 and the mix, which write the panels of every output bra sector)
// ---------------------------------------------------------------------------
struct EnvTab {
  int ng = 0, nPs = 0, nQs = 0, nRs = 0, nTs = 0;
  long long n1 = 0, npan = 0, nup = 0, ntmp = 0;
  Sec SP, SQ, SR, ST;
  std::vector<int> gcols, gld, Ntau, Ktau, t3tau, koff, pcol;
  std::vector<long long> goff, htmp, t3base, pbase, upoff, hbase;
  std::vector<EnvS1> s1;
  std::vector<int4> t1, tm, th, t3;
  std::vector<EnvUP> ups;
  std::vector<EnvS3> s3;
  DevMem d_s1, d_t1, d_cinfo, d_goff, d_gcols, d_specoff, d_th, d_hbase, d_nR, d_grp, d_spec, d_tm, d_t3tau, d_t3base,
      d_Ntau, d_pcol, d_ups, d_oP, d_nP, d_oT, d_nT, d_s3, d_t3;
  // heavy-row GEMMs of the mix, uploaded for the T1 and staging buffers they were built for
  std::vector<GemmGroup<double>> gg;
  DevMem ggdev;
  const double* gg_t1 = nullptr;
  const double* gg_tmp = nullptr;
};

// lP/lQ: bra/ket labels at the input bond, lR/lT: ket/bra labels at the output bond;
// Pp..Tp their padded sizes; ket_rrp: padded right bond of the ket core (its row stride).
static bool env_tab(Engine& E, const BsSiteUse& u, const Labels& lP, const Labels& lQ, const Labels& lR,
                    const Labels& lT, int Pp, int Qp, int Rp, int Tp, int ket_rrp, EnvTab& t) {
  (void)Pp; (void)Qp; (void)Rp; (void)Tp;
  const bool left = u.sigma > 0;
  const int sg = u.sigma;
  Sec &SP = t.SP, &SQ = t.SQ, &SR = t.SR, &ST = t.ST;
  if (!sectors(lP, SP) || !sectors(lQ, SQ) || !sectors(lR, SR) || !sectors(lT, ST)) return false;
  const int nPs = (int)SP.q.size(), nQs = (int)SQ.q.size(), nRs = (int)SR.q.size(), nTs = (int)ST.q.size();
  t.nPs = nPs; t.nQs = nQs; t.nRs = nRs; t.nTs = nTs;
  const int ng = u.ngrp;
  t.ng = ng;

  // spectators (pi, rho) grouped by Gamma = Q_rho - Q_pi
  std::vector<int>& gcols = t.gcols;
  gcols.assign(ng, 0);
  std::vector<std::vector<int4>> spec_g(ng);
  std::vector<long long> specoff((size_t)std::max(nPs * nRs, 1), -1);
  for (int pi = 0; pi < nPs; ++pi)
    for (int rho = 0; rho < nRs; ++rho) {
      auto it = u.gid.find(sub(SR.q[rho], SP.q[pi]));
      if (it == u.gid.end()) continue;
      const int g = it->second;
      specoff[(size_t)pi * nRs + rho] = gcols[g];
      spec_g[g].push_back(make_int4(gcols[g], pi, rho, 0));
      gcols[g] += SP.n[pi] * SR.n[rho];
    }
  // T1 rows of a group are stored with a stride rounded up to 4 elements
  t.goff.assign(ng, 0);
  t.gld.assign(ng, 0);
  long long n1 = 0;
  std::vector<int4> spec;
  std::vector<EnvGrp> grp(ng);
  for (int g = 0; g < ng; ++g) {
    t.gld[g] = (gcols[g] + 3) / 4 * 4;
    t.goff[g] = n1;
    n1 += (long long)u.nrows_in[g] * t.gld[g];
    grp[g] = EnvGrp{t.goff[g], gcols[g], (int)spec.size(), (int)spec_g[g].size(), t.gld[g]};
    spec.insert(spec.end(), spec_g[g].begin(), spec_g[g].end());
  }
  t.n1 = n1;

  // stage 1: per (input class c, ket sector kappa)
  std::vector<int4> cinfo;
  std::vector<int> col0(nQs), ncol(nQs);
  for (int ka = 0; ka < nQs; ++ka) {
    col0[ka] = (int)cinfo.size();
    for (int s = 0; s < 4; ++s) {
      const int rho = SR.find(add(SQ.q[ka], mul(sg, kQ[s])));
      if (rho < 0) continue;
      for (int ir = 0; ir < SR.n[rho]; ++ir) {
        const int cx = left ? s * ket_rrp + SR.off[rho] + ir : (SR.off[rho] + ir) * 4 * ket_rrp + s * ket_rrp;
        cinfo.push_back(make_int4(cx, s, rho, ir));
      }
    }
    ncol[ka] = (int)cinfo.size() - col0[ka];
  }
  for (int c = 0; c < u.ncin; ++c) {
    const int cnt = u.cstart_in[c + 1] - u.cstart_in[c];
    for (int ka = 0; ka < nQs; ++ka) {
      const int pi = SP.find(add(SQ.q[ka], u.cq_in[c]));
      if (pi < 0 || ncol[ka] == 0 || cnt == 0) continue;
      EnvS1 d{cnt * SP.n[pi], ncol[ka], SQ.n[ka], u.cstart_in[c], SP.n[pi], SP.off[pi], SQ.off[ka], col0[ka], pi, 0};
      const int id = (int)t.s1.size();
      t.s1.push_back(d);
      for (int m0 = 0; m0 < d.M; m0 += TL)
        for (int c0 = 0; c0 < d.N; c0 += TL) t.t1.push_back(make_int4(id, m0, c0, 0));
    }
  }

  // panels: tau rows (pi, s', i_p) with Q_tau = Q_pi + sigma q(s'); columns (class c', K', i_r)
  t.Ntau.assign(nTs, 0);
  t.Ktau.assign(nTs, 0);
  t.pcol.assign((size_t)std::max(nTs * u.ncout, 1), -1);
  for (int ta = 0; ta < nTs; ++ta)
    for (int c = 0; c < u.ncout; ++c) {
      const int rho = SR.find(sub(ST.q[ta], u.cq_out[c]));
      if (rho < 0) continue;
      t.pcol[(size_t)ta * u.ncout + c] = t.Ntau[ta];
      t.Ntau[ta] += (u.cstart_out[c + 1] - u.cstart_out[c]) * SR.n[rho];
    }
  t.t3tau.assign((size_t)std::max(nPs * 4, 1), -1);
  t.koff.assign((size_t)std::max(nPs * 4, 1), 0);
  for (int ta = 0; ta < nTs; ++ta)
    for (int pi = 0; pi < nPs; ++pi)
      for (int s = 0; s < 4; ++s)
        if (add(SP.q[pi], mul(sg, kQ[s])) == ST.q[ta]) {
          t.t3tau[pi * 4 + s] = ta;
          t.koff[pi * 4 + s] = t.Ktau[ta];
          t.Ktau[ta] += SP.n[pi];
        }
  t.pbase.assign(nTs, 0);
  t.upoff.assign(nTs, 0);
  long long npan = 0, nup = 0;
  for (int ta = 0; ta < nTs; ++ta) {
    t.pbase[ta] = npan;
    npan += (long long)t.Ktau[ta] * t.Ntau[ta];
    t.upoff[ta] = nup;
    nup += (long long)ST.n[ta] * t.Ktau[ta];
  }
  t.npan = npan;
  t.nup = nup;
  t.t3base.assign((size_t)std::max(nPs * 4, 1), -1);
  for (int pi = 0; pi < nPs; ++pi)
    for (int s = 0; s < 4; ++s) {
      const int ta = t.t3tau[pi * 4 + s];
      if (ta < 0) continue;
      t.t3base[pi * 4 + s] = t.pbase[ta] + (long long)t.koff[pi * 4 + s] * t.Ntau[ta];
      t.ups.push_back(EnvUP{t.upoff[ta], ta, pi, s, t.koff[pi * 4 + s], t.Ktau[ta], 0});
    }

  // mix tiles: light rows, and heavy rows (staged by the GEMM) with their staging offsets
  t.hbase.assign((size_t)std::max(u.hrow0[ng], 1), 0);
  t.htmp.assign(ng, 0);
  long long ntmp = 0;
  for (int g = 0; g < ng; ++g) {
    if (gcols[g] == 0) continue;
    for (int c0 = 0; c0 < gcols[g]; c0 += MC)
      for (int r0 = u.orow0[g]; r0 < u.orow0[g + 1]; r0 += MR)
        t.tm.push_back(make_int4(g, c0, r0, std::min(r0 + MR, u.orow0[g + 1])));
    if (u.hrow0[g + 1] > u.hrow0[g]) {
      t.htmp[g] = ntmp;
      for (int r = u.hrow0[g]; r < u.hrow0[g + 1]; ++r) t.hbase[r] = ntmp + (long long)(r - u.hrow0[g]) * t.gld[g];
      ntmp += (long long)(u.hrow0[g + 1] - u.hrow0[g]) * t.gld[g];
      for (int c0 = 0; c0 < gcols[g]; c0 += MC)
        for (int r0 = u.hrow0[g]; r0 < u.hrow0[g + 1]; r0 += MR)
          t.th.push_back(make_int4(g, c0, r0, std::min(r0 + MR, u.hrow0[g + 1])));
    }
  }
  t.ntmp = ntmp;

  // stage 3: per (tau, output class c')
  for (int ta = 0; ta < nTs; ++ta) {
    if (t.Ktau[ta] == 0) continue;
    for (int c = 0; c < u.ncout; ++c) {
      const int pc = t.pcol[(size_t)ta * u.ncout + c];
      if (pc < 0) continue;
      const int rho = SR.find(sub(ST.q[ta], u.cq_out[c]));
      const int cnt = u.cstart_out[c + 1] - u.cstart_out[c];
      EnvS3 d{t.upoff[ta], t.pbase[ta], ST.n[ta], cnt * SR.n[rho], t.Ktau[ta], t.Ntau[ta], pc, u.cstart_out[c],
              SR.n[rho], SR.off[rho], ST.off[ta], 0};
      const int id = (int)t.s3.size();
      t.s3.push_back(d);
      for (int m0 = 0; m0 < d.M; m0 += TL)
        for (int n0 = 0; n0 < d.N; n0 += TL) t.t3.push_back(make_int4(id, m0, n0, 0));
    }
  }

  // device tables
  hipStream_t st = E.stream;
  up(t.d_s1, t.s1, st);
  up(t.d_t1, t.t1, st);
  up(t.d_cinfo, cinfo, st);
  up(t.d_goff, t.goff, st);
  up(t.d_gcols, t.gld, st);
  up(t.d_th, t.th, st);
  up(t.d_hbase, t.hbase, st);
  up(t.d_specoff, specoff, st);
  up(t.d_nR, SR.n, st);
  up(t.d_grp, grp, st);
  up(t.d_spec, spec, st);
  up(t.d_tm, t.tm, st);
  up(t.d_t3tau, t.t3tau, st);
  up(t.d_t3base, t.t3base, st);
  up(t.d_Ntau, t.Ntau, st);
  up(t.d_pcol, t.pcol, st);
  up(t.d_ups, t.ups, st);
  up(t.d_oP, SP.off, st);
  up(t.d_nP, SP.n, st);
  up(t.d_oT, ST.off, st);
  up(t.d_nT, ST.n, st);
  up(t.d_s3, t.s3, st);
  up(t.d_t3, t.t3, st);
  return true;
}

// stage 1 and the mix: T1 (n1 elements, zeroed here), the panels (npan), the heavy-row
// staging buffer tmp (ntmp).  Ein: [nin][Pp][Qp]; ket: the ket core (nket elements).
static void env_panel(Engine& E, const BsSiteUse& u, EnvTab& t, const double* Ein, long long nE, int Qp,
                      long long PQ, const double* ket, long long nket, long long bks, double* T1, double* panel,
                      double* tmp, int* err, bool timed = false) {
  // timed: per-kernel events of a product (slots 0 stage 1, 1 light mix, 2 heavy GEMM, 3 heavy mix)
  auto mark = [&](int slot) {
    if (timed) E.kt_mark(slot);
  };
  hipStream_t st = E.stream;
  // T1 entries whose ket sector Q_pi - d_K does not exist are never written
  fill(T1, sizeof(double) * t.n1, st);
  if (!t.t1.empty()) {
    hipLaunchKernelGGL(env_s1_kernel, dim3((unsigned)t.t1.size()), dim3(256), 0, st, t.d_t1.as<int4>(),
                       t.d_s1.as<EnvS1>(), u.clist_in.as<int>(), t.d_cinfo.as<int4>(), u.d_gidx_in.as<int>(),
                       u.rin.as<int>(), t.d_goff.as<long long>(), t.d_gcols.as<int>(), t.d_specoff.as<long long>(),
                       t.d_nR.as<int>(), t.nRs, Ein, PQ, Qp, nE, ket, nket, bks, T1, t.n1, err);
    BECHECK(hipGetLastError());
    mark(0);
  }
  if (!t.tm.empty()) {
    hipLaunchKernelGGL(env_mix_kernel, dim3((unsigned)t.tm.size()), dim3(MC), 0, st, t.d_tm.as<int4>(),
                       t.d_grp.as<EnvGrp>(), u.optr.as<int>(), u.ocol.as<int>(), u.oval.as<double>(),
                       u.orow.as<int2>(), t.d_spec.as<int4>(), T1, t.n1, panel, t.npan, t.d_t3tau.as<int>(),
                       t.d_t3base.as<long long>(), t.d_Ntau.as<int>(), t.d_pcol.as<int>(), u.ncout,
                       u.d_cls_out.as<int>(), u.pos_out.as<int>(), t.d_nR.as<int>(), err,
                       (const long long*)nullptr, (const double*)nullptr);
    BECHECK(hipGetLastError());
    mark(1);
  }
  if (!t.th.empty()) {
    if (t.gg_t1 != T1 || t.gg_tmp != tmp) {
      t.gg.clear();
      for (int g = 0; g < t.ng; ++g) {
        const int H = u.hrow0[g + 1] - u.hrow0[g];
        if (H == 0 || t.gcols[g] == 0) continue;
        GemmGroup<double> G{};
        G.g.M = H; G.g.N = t.gcols[g]; G.g.K = u.nrows_in[g]; G.g.batch = 1;
        G.g.kin = std::max(16, (u.nrows_in[g] + 15) / 16 * 16);
        G.g.sAm = u.nin4[g]; G.g.sAkk = 1;
        G.g.sBkk = t.gld[g]; G.g.sBn = 1;
        G.g.sCm = t.gld[g]; G.g.alpha = 1.0; G.g.beta = 0.0;
        G.A = u.hw.as<double>() + u.hw_off[g];
        G.B = T1 + t.goff[g];
        G.C = tmp + t.htmp[g];
        t.gg.push_back(G);
      }
      upload(t.ggdev, t.gg.data(), t.gg.size() * sizeof(GemmGroup<double>), st);
      t.gg_t1 = T1;
      t.gg_tmp = tmp;
    }
    gemm_grouped<double>(t.ggdev.as<GemmGroup<double>>(), t.gg, st);
    mark(2);
    hipLaunchKernelGGL(env_mix_kernel, dim3((unsigned)t.th.size()), dim3(MC), 0, st, t.d_th.as<int4>(),
                       t.d_grp.as<EnvGrp>(), u.optr.as<int>(), u.ocol.as<int>(), u.oval.as<double>(),
                       u.hrow.as<int2>(), t.d_spec.as<int4>(), T1, t.n1, panel, t.npan, t.d_t3tau.as<int>(),
                       t.d_t3base.as<long long>(), t.d_Ntau.as<int>(), t.d_pcol.as<int>(), u.ncout,
                       u.d_cls_out.as<int>(), u.pos_out.as<int>(), t.d_nR.as<int>(), err, t.d_hbase.as<long long>(),
                       (const double*)tmp);
    BECHECK(hipGetLastError());
    mark(3);
  }
}

static void check_err(DevMem& d_err, hipStream_t st, const char* what) {
  int herr = 0;
  BECHECK(hipMemcpyAsync(&herr, d_err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  BECHECK(hipStreamSynchronize(st));
  if (herr != 0)
    throw std::runtime_error(std::string(what) + ": index outside its buffer (check " + std::to_string(herr) + ")");
}

// ---------------------------------------------------------------------------
// one update
// ---------------------------------------------------------------------------
bool bs_env(Engine& E, const BsSiteUse& u, const double* Ein, const Core& bra, const Core& ket, double* out) {
  const bool left = u.sigma > 0;
  const Labels& lP = left ? bra.ql : bra.qr;
  const Labels& lQ = left ? ket.ql : ket.qr;
  const Labels& lR = left ? ket.qr : ket.ql;
  const Labels& lT = left ? bra.qr : bra.ql;
  if ((int)bra.ql.size() != bra.rl || (int)bra.qr.size() != bra.rr || (int)ket.ql.size() != ket.rl ||
      (int)ket.qr.size() != ket.rr)
    return false;
  const int Pp = left ? bra.rlp() : bra.rrp(), Qp = left ? ket.rlp() : ket.rrp();
  const int Rp = left ? ket.rrp() : ket.rlp(), Tp = left ? bra.rrp() : bra.rlp();
  EnvTab t;
  if (!env_tab(E, u, lP, lQ, lR, lT, Pp, Qp, Rp, Tp, ket.rrp(), t)) return false;
  hipStream_t st = E.stream;
  DevMem d_err;
  d_err.resize_zero(sizeof(int), st);
  int* err = d_err.as<int>();
  E.be_t1.ensure(sizeof(double) * std::max<long long>(t.n1, 1));
  E.be_panel.ensure(sizeof(double) * std::max<long long>(t.npan, 1));
  E.be_up.ensure(sizeof(double) * std::max<long long>(t.nup, 1));
  if (!t.th.empty()) E.be_tmp.ensure(sizeof(double) * std::max<long long>(t.ntmp, 1));
  const long long nE = (long long)u.nin * Pp * Qp;
  const long long nout = (long long)u.nout * Tp * Rp;
  const long long nket = (long long)ket.rlp() * 4 * ket.rrp();
  const long long nbra = (long long)bra.rlp() * 4 * bra.rrp();
  fill(out, sizeof(double) * nout, st);
  const long long bks = left ? 4LL * ket.rrp() : 1LL;
  env_panel(E, u, t, Ein, nE, Qp, (long long)Pp * Qp, ket.d.as<double>(), nket, bks, E.be_t1.as<double>(),
            E.be_panel.as<double>(), t.th.empty() ? nullptr : E.be_tmp.as<double>(), err);
  if (!t.ups.empty()) {
    const long long rbp = bra.rrp();
    const long long ps = left ? 4 * rbp : 1, ss = rbp, ts = left ? 1 : 4 * rbp;
    hipLaunchKernelGGL(env_up_kernel, dim3((unsigned)t.ups.size()), dim3(256), 0, st, t.d_ups.as<EnvUP>(),
                       bra.d.as<double>(), nbra, ps, ss, ts, t.d_oP.as<int>(), t.d_nP.as<int>(), t.d_oT.as<int>(),
                       t.d_nT.as<int>(), E.be_up.as<double>(), t.nup, err);
    BECHECK(hipGetLastError());
  }
  if (!t.t3.empty()) {
    hipLaunchKernelGGL(env_s3_kernel, dim3((unsigned)t.t3.size()), dim3(256), 0, st, t.d_t3.as<int4>(),
                       t.d_s3.as<EnvS3>(), E.be_up.as<double>(), t.nup, E.be_panel.as<double>(), t.npan,
                       u.clist_out.as<int>(), out, nout, (long long)Tp * Rp, Rp, err);
    BECHECK(hipGetLastError());
  }
  check_err(d_err, st, "block-sparse environment update");
  return true;
}

// ---------------------------------------------------------------------------
// one-site effective-Hamiltonian product (eq. mat_vec, one-site form)
//   y[a'][s'][b'] = sum L[A][a'][a] W[A,s',s,B] x[a][s][b] R[B][b'][b]
// Stage 1 and the mix of the left update with ket = x leave, for every output
// bra sector tau of the right bond, the panel P_tau[(pi, s', i_p)][(B, i_r)] =
// sum L W x.  The last stage multiplies it by the right environment stacked per
// tau, Rs_tau[(B, i_r)][j] = R[B][o_tau + j][o_rho + i_r] (built once per local
// problem): the split-K MFMA tiles of the two-site product's last stage over each
// tau's whole panel, whose K chunks are summed and scattered into the rows of y.
// ---------------------------------------------------------------------------
namespace {
struct R1Desc { long long dst; int cls0, cnt, nr, orho, ntau, otau, pad; };

__global__ __launch_bounds__(256) void rstack1_kernel(const R1Desc* __restrict__ desc,
                                                      const int* __restrict__ clist_out,
                                                      const double* __restrict__ R, long long nR, int rrp,
                                                      double* __restrict__ Rs, long long nRs, int* __restrict__ err) {
  const R1Desc d = desc[blockIdx.x];
  const long long tot = (long long)d.cnt * d.nr * d.ntau;
  for (long long e = threadIdx.x; e < tot; e += 256) {
    const int j = (int)(e % d.ntau);
    const long long row = e / d.ntau;
    const int ir = (int)(row % d.nr), pos = (int)(row / d.nr);
    const int K = clist_out[d.cls0 + pos];
    const long long q = ((long long)K * rrp + d.otau + j) * rrp + d.orho + ir;
    const long long dst = d.dst + e;
    if (q < 0 || q >= nR || dst < 0 || dst >= nRs) { err[0] = 21; continue; }
    Rs[dst] = R[q];
  }
}
}  // namespace

struct BsHeff1Impl {
  EnvTab t;
  std::shared_ptr<BsSiteUse> use;
  int rlp = 0, rrp = 0, RAx = 0;
  DevMem t1, panel, tmp, Rs, err;
  std::vector<long long> rsoff;
  // last stage: split-K tiles over the panels of every right sector, rows scattered into y
  int ntiles = 0, nred = 0, nslots = 0;
  long long nrs = 0;
  DevMem tiles, red, rowdst, part;
  double kfl[TT_KT_SLOTS] = {}, kby[TT_KT_SLOTS] = {};  // algorithmic flops and bytes per timing slot
};

bool bs_heff1_build(Engine& E, BsHeff1& h, std::shared_ptr<BsSiteUse> use, const Labels& ql, const Labels& qr, int RAx,
                    const double* R, int RB) {
  auto p = std::make_shared<BsHeff1Impl>();
  const BsSiteUse& u = *use;
  if (u.sigma != 1 || u.nin != RAx || u.nout != RB)
    throw std::runtime_error("one-site product: site tables do not match the environments");
  p->use = use;
  p->RAx = RAx;
  p->rlp = padr((int)ql.size());
  p->rrp = padr((int)qr.size());
  // bra = ket = x: P = Q = left bond labels, R = T = right bond labels
  if (!env_tab(E, u, ql, ql, qr, qr, p->rlp, p->rlp, p->rrp, p->rrp, p->rrp, p->t)) return false;
  EnvTab& t = p->t;
  hipStream_t st = E.stream;
  p->t1.ensure(sizeof(double) * std::max<long long>(t.n1, 1));
  p->panel.ensure(sizeof(double) * std::max<long long>(t.npan, 1));
  if (!t.th.empty()) p->tmp.ensure(sizeof(double) * std::max<long long>(t.ntmp, 1));
  p->err.resize_zero(sizeof(int), st);
  // stacked right environment per tau: rows = panel columns (class, K', i_r), columns j
  std::vector<R1Desc> rd;
  p->rsoff.assign(t.nTs, 0);
  long long nrs = 0;
  for (int ta = 0; ta < t.nTs; ++ta) {
    p->rsoff[ta] = nrs;
    const int ntau = t.ST.n[ta];
    for (int c = 0; c < u.ncout; ++c) {
      const int pc = t.pcol[(size_t)ta * u.ncout + c];
      if (pc < 0) continue;
      const int rho = t.SR.find(sub(t.ST.q[ta], u.cq_out[c]));
      const int cnt = u.cstart_out[c + 1] - u.cstart_out[c];
      if (cnt == 0 || t.SR.n[rho] == 0 || ntau == 0) continue;
      rd.push_back(R1Desc{nrs + (long long)pc * ntau, u.cstart_out[c], cnt, t.SR.n[rho], t.SR.off[rho], ntau,
                          t.ST.off[ta], 0});
    }
    nrs += (long long)t.Ntau[ta] * ntau;
  }
  p->nrs = nrs;
  p->Rs.resize_zero(sizeof(double) * std::max<long long>(nrs, 1), st);
  if (!rd.empty()) {
    DevMem d_rd;
    up(d_rd, rd, st);
    hipLaunchKernelGGL(rstack1_kernel, dim3((unsigned)rd.size()), dim3(256), 0, st, d_rd.as<R1Desc>(),
                       u.clist_out.as<int>(), R, (long long)RB * p->rrp * p->rrp, p->rrp, p->Rs.as<double>(),
                       std::max<long long>(nrs, 1), p->err.as<int>());
    BECHECK(hipGetLastError());
    check_err(p->err, st, "one-site product set-up");
  }
  // last stage: one split-K segment per right sector tau (panel [Ktau][Ntau] x stacked
  // R [Ntau][n_tau]); panel row koff(pi, s') + i_p is y row (o_pi + i_p, s'), columns o_tau..
  std::vector<BsSplitSeg> segs;
  std::vector<long long> rowdst;
  std::vector<long long> row0(t.nTs, 0);
  for (int ta = 0; ta < t.nTs; ++ta) {
    row0[ta] = (long long)rowdst.size();
    rowdst.resize(rowdst.size() + t.Ktau[ta], -1);
    segs.push_back(BsSplitSeg{t.pbase[ta], p->rsoff[ta], t.Ktau[ta], t.ST.n[ta], t.Ntau[ta], (int)row0[ta]});
  }
  for (const EnvUP& e : t.ups)
    for (int i = 0; i < t.SP.n[e.pi]; ++i)
      rowdst[row0[e.tau] + e.koff + i] = (((long long)t.SP.off[e.pi] + i) * 4 + e.s) * p->rrp + t.ST.off[e.tau];
  for (long long d : rowdst)
    if (d < 0) throw std::runtime_error("one-site product: a panel row has no destination");
  std::vector<BsS4Tile> tiles;
  std::vector<BsRedTile> red;
  double el_red = 0.0;
  bs_splitk_tables(segs, tiles, red, p->nslots, el_red);
  p->ntiles = (int)tiles.size();
  p->nred = (int)red.size();
  up(p->tiles, tiles, st);
  up(p->red, red, st);
  up(p->rowdst, rowdst, st);
  p->part.ensure(sizeof(double) * (size_t)std::max(p->nslots, 1) * kBsSplitTile * kBsSplitTile);
  // algorithmic work per timing slot (quantum-number-allowed blocks, each operand
  // element moved once): 0 stage 1, 1 light mix, 2 heavy GEMM, 3 heavy mix, 7 last
  // stage's products, 8 their K-split reduction
  double* kf = p->kfl;
  double* kb = p->kby;
  for (const EnvS1& d : t.s1) {
    kf[0] += 2.0 * d.M * (double)d.N * d.K;
    kb[0] += 8.0 * ((double)d.M * d.K + (double)d.K * d.N + (double)d.M * d.N);
  }
  for (int g = 0; g < t.ng; ++g) {
    const double cols = t.gcols[g];
    const double nl = u.orow0[g + 1] - u.orow0[g], H = u.hrow0[g + 1] - u.hrow0[g], nin = u.nrows_in[g];
    kf[1] += 2.0 * u.nent_light[g] * cols;
    kb[1] += 8.0 * cols * ((nl > 0 ? nin : 0.0) + nl);
    if (H > 0) {
      kf[2] += 2.0 * H * nin * cols;
      kb[2] += 8.0 * (H * nin + nin * cols + H * cols);
      kb[3] += 8.0 * 2.0 * H * cols;
    }
  }
  for (int ta = 0; ta < t.nTs; ++ta) {
    const double M = t.Ktau[ta], K = t.Ntau[ta], N = t.ST.n[ta];
    kf[7] += 2.0 * M * K * N;
    kb[7] += 8.0 * (M * K + K * N + M * N);
  }
  kb[8] = 8.0 * el_red;
  h.flops = kf[0] + kf[1] + kf[2] + kf[7];
  h.p = p;
  return true;
}

void bs_heff1_apply(Engine& E, BsHeff1& h, const double* Lx, const double* x, double* y) {
  BsHeff1Impl& p = *h.p;
  EnvTab& t = p.t;
  const BsSiteUse& u = *p.use;
  hipStream_t st = E.stream;
  const long long nx = (long long)p.rlp * 4 * p.rrp;
  fill(y, sizeof(double) * nx, st);
  E.kt_begin();
  env_panel(E, u, t, Lx, (long long)p.RAx * p.rlp * p.rlp, p.rlp, (long long)p.rlp * p.rlp, x, nx, 4LL * p.rrp,
            p.t1.as<double>(), p.panel.as<double>(), t.th.empty() ? nullptr : p.tmp.as<double>(), p.err.as<int>(),
            true);
  bs_splitk_run(E, p.ntiles, p.tiles.as<BsS4Tile>(), p.nred, p.red.as<BsRedTile>(), p.rowdst.as<long long>(),
                p.panel.as<double>(), std::max<long long>(t.npan, 1), p.Rs.as<double>(), std::max<long long>(p.nrs, 1),
                p.part.as<double>(), y, nx, p.err.as<int>(), 7, 8);
  check_err(p.err, st, "one-site product");
  E.kt_end(p.kfl, p.kby);
}

}  // namespace tt
