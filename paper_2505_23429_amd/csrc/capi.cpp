// C ABI (include/tt.h) over the engine.  No exception crosses this boundary.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>
#include <new>
#include <stdexcept>
#include <string>

#include "engine.h"

using tt::Engine;

namespace {

// the context's allocator and stream for the blocks this thread allocates during one call
struct CallAllocator {
  explicit CallAllocator(Engine& E) { tt::set_thread_allocator(&E.ext, E.stream); }
  ~CallAllocator() { tt::set_thread_allocator(nullptr, nullptr); }
};

template <class F>
int guard(void* ctx, F&& f) {
  Engine* E = static_cast<Engine*>(ctx);
  if (!E) return TT_EINVAL;
  CallAllocator scope(*E);
  try {
    E->err.clear();
    return f(*E);
  } catch (const std::invalid_argument& e) {
    E->err = e.what();
    return TT_EINVAL;
  } catch (const std::logic_error& e) {
    E->err = e.what();
    return TT_ESTATE;
  } catch (const std::bad_alloc&) {
    E->err = "host allocation failed";
    return TT_ENOMEM;
  } catch (const tt::DeviceOOM& e) {
    E->err = e.what();
    return TT_ENOMEM;
  } catch (const tt::HipError& e) {
    E->err = e.what();
    return TT_EHIP;
  } catch (const tt::SolverError& e) {
    E->err = e.what();
    return TT_EHIP;
  } catch (const std::exception& e) {
    E->err = e.what();
    return TT_EINTERNAL;
  } catch (...) {
    E->err = "unknown error";
    return TT_EINTERNAL;
  }
}

void check_entries(int nnz, const int32_t* A, const int32_t* B, int RA, int RB) {
  if (nnz < 0) throw std::invalid_argument("negative nnz");
  for (int e = 0; e < nnz; ++e)
    if (A[e] < 0 || A[e] >= RA || B[e] < 0 || B[e] >= RB) throw std::invalid_argument("MPO entry index out of range");
}

std::vector<int> vec(const int32_t* p, int n) { return std::vector<int>(p, p + n); }

}  // namespace

namespace {
// one table or workspace carved from the no-allocation scratch (256-byte aligned)
struct Carve {
  char* base;
  size_t off = 0;
  template <class T> T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off += (count * sizeof(T) + 255) / 256 * 256;
    return p;
  }
};

template <class T>
int heff_noalloc(Engine& E, int rl, int rr, int RA, int RB, int RC, const T* Lenv, const T* Renv, int nnz1,
                 const int32_t* A1, const int32_t* B1, const double* ops1, int nnz2, const int32_t* A2,
                 const int32_t* B2, const double* ops2, const T* x, T* y) {
  std::vector<int> p1, s1, p2, s2;
  std::vector<double> o64a, o64b;
  std::vector<float> o32a, o32b;
  tt::siteop_csr(RB, vec(B1, nnz1), vec(A1, nnz1), std::vector<double>(ops1, ops1 + 16LL * nnz1), p1, s1, o64a, o32a);
  tt::siteop_csr(RC, vec(B2, nnz2), vec(A2, nnz2), std::vector<double>(ops2, ops2 + 16LL * nnz2), p2, s2, o64b, o32b);
  const size_t slab = (size_t)rl * 16 * rr;
  // the byte count of the carve below, checked before anything is written
  auto rnd = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t need = rnd(p1.size() * 4) + rnd(s1.size() * 4) + rnd(o64a.size() * sizeof(T)) + rnd(p2.size() * 4) +
                      rnd(s2.size() * 4) + rnd(o64b.size() * sizeof(T)) +
                      rnd(slab * std::max(RA, RC) * sizeof(T)) + rnd(slab * RB * sizeof(T));
  if (need > tt::kNoallocScratchBytes)
    throw std::invalid_argument("tt_heff_apply_dev_noalloc: the product needs " + std::to_string(need) +
                                " bytes of scratch, more than its fixed " +
                                std::to_string(tt::kNoallocScratchBytes) + " bytes (use tt_heff_apply_dev)");
  Carve c{static_cast<char*>(E.noalloc)};
  int* d_p1 = c.take<int>(p1.size());
  int* d_s1 = c.take<int>(s1.size());
  T* d_o1 = c.take<T>(o64a.size());
  int* d_p2 = c.take<int>(p2.size());
  int* d_s2 = c.take<int>(s2.size());
  T* d_o2 = c.take<T>(o64b.size());
  T* ws_a = c.take<T>(slab * std::max(RA, RC));
  T* ws_b = c.take<T>(slab * RB);
  auto h2d = [&](void* d, const void* h, size_t bytes) {
    if (hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, E.stream) != hipSuccess)
      throw tt::HipError("HIP: copy into the no-allocation scratch failed");
  };
  h2d(d_p1, p1.data(), p1.size() * 4);
  h2d(d_s1, s1.data(), s1.size() * 4);
  h2d(d_p2, p2.data(), p2.size() * 4);
  h2d(d_s2, s2.data(), s2.size() * 4);
  if (sizeof(T) == 8) {
    h2d(d_o1, o64a.data(), o64a.size() * 8);
    h2d(d_o2, o64b.data(), o64b.size() * 8);
  } else {
    h2d(d_o1, o32a.data(), o32a.size() * 4);
    h2d(d_o2, o32b.data(), o32b.size() * 4);
  }
  tt::heff_dense<T>(E, rl, rr, RA, Lenv, RB, d_p1, d_s1, d_o1, RC, d_p2, d_s2, d_o2, Renv, x, y, ws_a, ws_b, nullptr,
                    0, 0, nullptr, false);
  // the host tables above must outlive their copies
  if (hipStreamSynchronize(E.stream) != hipSuccess) throw tt::HipError("HIP: stream synchronisation failed");
  return TT_OK;
}
}  // namespace

extern "C" {

void tt_default_opts(tt_opts* o) {
  if (!o) return;
  o->chi_max = 64;
  o->svd_cutoff = 1e-12;
  o->tie_rel = 1e-10;
  o->dav_tol = 1e-8;
  o->dav_maxiter = 200;
  o->dav_maxsub = 24;
  o->coarse_eps = 1e-8;
  o->matvec_prec = TT_F64;
  o->refine_fp64 = 0;
  o->lowprec_tol = 1e-5;
  o->device = 0;
  o->qn_skip = 1;
  o->sub_workers = 0;
  o->mix_stage = 0;
  o->svd_lds = 1;
  o->worker_alloc_limit = 0;
  o->stream = nullptr;
  o->dev_alloc = nullptr;
  o->dev_free = nullptr;
  o->alloc_user = nullptr;
  o->coarse_k = 1;
  o->one_site = 0;
  o->functional = 0;
  o->coarse_krylov = 0;
  o->graph_products = 0;
  o->precontract = 2;
  o->svd_blocked = 1;
}

int tt_create(const tt_opts* opts, void** out) {
  if (!opts || !out) return TT_EINVAL;
  *out = nullptr;
  if (opts->chi_max <= 0 || opts->dav_maxiter <= 0 || opts->dav_maxsub < 4 || opts->matvec_prec < 0 ||
      opts->matvec_prec > 2 || opts->sub_workers < 0 || opts->sub_workers > TT_MAX_SUB ||
      opts->mix_stage < 0 || opts->mix_stage > 2 || opts->svd_lds < 0 || opts->svd_lds > 1 ||
      opts->worker_alloc_limit < 0 || (!opts->dev_alloc) != (!opts->dev_free) || opts->coarse_k < 1 ||
      opts->coarse_k > 8 || opts->one_site < 0 || opts->one_site > 1 ||
      (opts->one_site && (opts->matvec_prec != TT_F64 || !opts->qn_skip)) || opts->functional < 0 ||
      opts->functional > 1 ||
      (opts->functional == 1 && (opts->matvec_prec != TT_F64 || !opts->qn_skip || opts->coarse_k != 1)) ||
      opts->coarse_krylov < 0 || opts->coarse_krylov > 1 || (opts->coarse_krylov && opts->functional != 0) ||
      opts->graph_products < 0 || opts->graph_products > 1 || opts->precontract < 0 || opts->precontract > 2 ||
      opts->svd_blocked < 0 || opts->svd_blocked > 4)
    return TT_EINVAL;
  try {
    *out = new Engine(*opts);
    return TT_OK;
  } catch (const std::exception&) {
    return TT_EHIP;
  }
}

void tt_destroy(void* ctx) { delete static_cast<Engine*>(ctx); }

const char* tt_last_error(const void* ctx) {
  const Engine* E = static_cast<const Engine*>(ctx);
  return E ? E->err.c_str() : "null context";
}

int tt_set_mpo(void* ctx, int L, const int* R, const int* nnz, const int32_t* const* A, const int32_t* const* B,
               const double* const* ops, const int32_t* const* chan_q, const int* block) {
  return guard(ctx, [&](Engine& E) {
    if (!R || !nnz || !A || !B || !ops || !chan_q || L < 2) throw std::invalid_argument("bad MPO arguments");
    E.set_mpo(L, R, nnz, A, B, ops, chan_q, block);
    return TT_OK;
  });
}

int tt_set_mps(void* ctx, int L, const int* r, const double* const* U, const int32_t* const* q) {
  return guard(ctx, [&](Engine& E) {
    if (!r || !U || !q) throw std::invalid_argument("bad TT arguments");
    E.set_mps(L, r, U, q);
    return TT_OK;
  });
}

int tt_get_mps(void* ctx, int* r, double* const* U, int32_t* const* q) {
  return guard(ctx, [&](Engine& E) {
    if (!r) throw std::invalid_argument("r is NULL");
    E.get_mps(r, U, q);
    return TT_OK;
  });
}

int tt_energy(void* ctx, double* En) {
  return guard(ctx, [&](Engine& E) {
    if (!En) throw std::invalid_argument("E is NULL");
    *En = E.energy();
    return TT_OK;
  });
}

int tt_set_rhs(void* ctx, int L, const int* r, const double* const* F, const int32_t* const* q) {
  return guard(ctx, [&](Engine& E) {
    if (!r || !F || !q) throw std::invalid_argument("bad TT arguments");
    E.set_rhs(L, r, F, q);
    return TT_OK;
  });
}

int tt_functional(void* ctx, double* J) {
  return guard(ctx, [&](Engine& E) {
    if (!J) throw std::invalid_argument("J is NULL");
    if (!E.have_mps) throw std::logic_error("no TT iterate");
    *J = E.functional_value();
    return TT_OK;
  });
}

int tt_local_solve(void* ctx, int nsub, const int* lengths, double* E_local, int* matvecs) {
  return guard(ctx, [&](Engine& E) {
    if (!lengths) throw std::invalid_argument("lengths is NULL");
    E.warn = 0;
    E.local_solve(nsub, lengths, E_local, matvecs);
    return E.warn;
  });
}

int tt_coarse_correct(void* ctx, double* S_out, double* A_out, double* coef_out, double* lambda_out, double* E_out,
                      int* rankS_out) {
  return guard(ctx, [&](Engine& E) {
    double disc = 0.0;
    return E.coarse_correct(S_out, A_out, coef_out, lambda_out, E_out, rankS_out, &disc);
  });
}

int tt_mps_checkpoint(void* ctx, int op) {
  return guard(ctx, [&](Engine& E) {
    E.checkpoint(op);
    return TT_OK;
  });
}

int tt_sweep(void* ctx, int nsub, const int* lengths, tt_sweep_report* out) {
  return guard(ctx, [&](Engine& E) {
    if (!lengths || !out) throw std::invalid_argument("NULL argument");
    if (nsub <= 0 || nsub > TT_MAX_SUB) throw std::invalid_argument("bad number of subdomains");
    std::memset(out, 0, sizeof(*out));
    out->nsub = nsub;
    E.warn = 0;
    E.flops_heff = 0.0;
    E.sec_heff = 0.0;
    for (double& v : E.ph) v = 0.0;
    auto t0 = std::chrono::steady_clock::now();
    out->E_before = E.functional_value();
    auto t1 = std::chrono::steady_clock::now();
    E.local_solve(nsub, lengths, out->E_local, out->matvecs);
    for (int j = 0; j < nsub; ++j) out->matvecs_f64[j] = E.subs[E.sub_base[j]].matvecs64;
    auto t2 = std::chrono::steady_clock::now();
    const int n = (int)E.subs.size() + 1;
    out->nstates = n;
    std::vector<double> S((size_t)n * n), A((size_t)n * n);
    int st = E.coarse_correct(S.data(), A.data(), out->coef, &out->lambda, &out->E_after, &out->rankS,
                              &out->discarded);
    if (E.opts.functional == 1)
      for (int i = 0; i < n && i < (int)E.coarse_b.size(); ++i) out->rhs[i] = E.coarse_b[i];
    out->coarse_matvecs = E.coarse_matvecs;
    auto t3 = std::chrono::steady_clock::now();
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        out->S[i * n + j] = S[(size_t)i * n + j];
        out->A[i * n + j] = A[(size_t)i * n + j];
      }
    // step 1 (LQ + environments) and step 2 (local solves) share local_solve;
    // steps 3-4 share coarse_correct
    out->seconds[0] = std::chrono::duration<double>(t1 - t0).count();
    out->seconds[1] = std::chrono::duration<double>(t2 - t1).count();
    out->seconds[2] = std::chrono::duration<double>(t3 - t2).count();
    out->seconds[3] = 0.0;
    out->flops_heff = E.flops_heff;
    out->seconds_heff = E.sec_heff;
    for (int i = 0; i < Engine::NPH; ++i) out->phase_seconds[i] = E.ph[i];
    return std::max(st, E.warn);
  });
}

int tt_dmrg2(void* ctx, int nsweeps, double* energies) {
  return guard(ctx, [&](Engine& E) {
    if (nsweeps <= 0) throw std::invalid_argument("nsweeps must be positive");
    E.warn = 0;
    E.dmrg2(nsweeps, energies);
    return E.warn;
  });
}

int tt_window_apply_dev(void* ctx, int b, int rl, int rr, const int32_t* ql, const int32_t* qr, const double* Lenv,
                        const double* Renv, int prec, const double* x, double* y) {
  return guard(ctx, [&](Engine& E) {
    E.window_apply(b, rl, rr, ql, qr, Lenv, Renv, prec, x, y);
    return TT_OK;
  });
}

int tt_heff_apply_dev(void* ctx, int prec, int rl, int rr, int RA, int RB, int RC, const void* Lenv, const void* Renv,
                      int nnz1, const int32_t* A1, const int32_t* B1, const double* ops1, int nnz2, const int32_t* A2,
                      const int32_t* B2, const double* ops2, const void* x, void* y) {
  return guard(ctx, [&](Engine& E) {
    if (rl <= 0 || rr <= 0 || rl % tt::PAD || rr % tt::PAD)
      throw std::invalid_argument("rl and rr must be positive multiples of 32");
    if (RA <= 0 || RB <= 0 || RC <= 0) throw std::invalid_argument("channel counts must be positive");
    if (!Lenv || !Renv || !x || !y || (nnz1 && (!A1 || !B1 || !ops1)) || (nnz2 && (!A2 || !B2 || !ops2)))
      throw std::invalid_argument("NULL pointer");
    check_entries(nnz1, A1, B1, RA, RB);
    check_entries(nnz2, A2, B2, RB, RC);
    tt::SiteOp w1, w2;
    Engine::build_siteop(w1, RB, vec(B1, nnz1), vec(A1, nnz1), std::vector<double>(ops1, ops1 + 16LL * nnz1),
                         E.stream);
    Engine::build_siteop(w2, RC, vec(B2, nnz2), vec(A2, nnz2), std::vector<double>(ops2, ops2 + 16LL * nnz2),
                         E.stream);
    if (prec == TT_F64)
      E.heff<double>(rl, rr, RA, (const double*)Lenv, w1, RB, w2, RC, (const double*)Renv, (const double*)x,
                     (double*)y, nullptr, 0, 0);
    else if (prec == TT_F32)
      E.heff<float>(rl, rr, RA, (const float*)Lenv, w1, RB, w2, RC, (const float*)Renv, (const float*)x, (float*)y,
                    nullptr, 0, 0);
    else if (prec == TT_BF16)
      E.heff_bf16(rl, rr, RA, (const uint16_t*)Lenv, w1, RB, w2, RC, (const uint16_t*)Renv, (const uint16_t*)x,
                  (float*)y, nullptr, 0, 0);
    else
      throw std::invalid_argument("unknown precision");
    if (hipStreamSynchronize(E.stream) != hipSuccess) throw tt::HipError("HIP: stream synchronisation failed");
    return TT_OK;
  });
}


int tt_heff_apply_dev_noalloc(void* ctx, int prec, int rl, int rr, int RA, int RB, int RC, const void* Lenv,
                              const void* Renv, int nnz1, const int32_t* A1, const int32_t* B1, const double* ops1,
                              int nnz2, const int32_t* A2, const int32_t* B2, const double* ops2, const void* x,
                              void* y) {
  return guard(ctx, [&](Engine& E) {
    if (rl <= 0 || rr <= 0 || rl % tt::PAD || rr % tt::PAD)
      throw std::invalid_argument("rl and rr must be positive multiples of 32");
    if (RA <= 0 || RB <= 0 || RC <= 0) throw std::invalid_argument("channel counts must be positive");
    if (!Lenv || !Renv || !x || !y || (nnz1 && (!A1 || !B1 || !ops1)) || (nnz2 && (!A2 || !B2 || !ops2)))
      throw std::invalid_argument("NULL pointer");
    check_entries(nnz1, A1, B1, RA, RB);
    check_entries(nnz2, A2, B2, RB, RC);
    if (prec == TT_F64)
      return heff_noalloc<double>(E, rl, rr, RA, RB, RC, (const double*)Lenv, (const double*)Renv, nnz1, A1, B1, ops1,
                                  nnz2, A2, B2, ops2, (const double*)x, (double*)y);
    if (prec == TT_F32)
      return heff_noalloc<float>(E, rl, rr, RA, RB, RC, (const float*)Lenv, (const float*)Renv, nnz1, A1, B1, ops1,
                                 nnz2, A2, B2, ops2, (const float*)x, (float*)y);
    throw std::invalid_argument("tt_heff_apply_dev_noalloc: precision must be TT_F64 or TT_F32");
  });
}

int tt_gemm_dev(void* ctx, int prec, int M, int N, int K, int batch, int kin, const long long* st, int a_kcontig,
                int b_ncontig, double alpha, double beta, const void* A, const void* B, void* Cm) {
  return guard(ctx, [&](Engine& E) {
    if (!st || !A || !B || !Cm) throw std::invalid_argument("NULL pointer");
    if (M < 0 || N < 0 || K < 0 || batch < 0) throw std::invalid_argument("negative size");
    tt::GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.batch = batch; g.kin = kin;
    g.sAb = st[0]; g.sAm = st[1]; g.sAkb = st[2]; g.sAkk = st[3];
    g.sBb = st[4]; g.sBkb = st[5]; g.sBkk = st[6]; g.sBn = st[7];
    g.sCb = st[8]; g.sCm = st[9]; g.alpha = alpha; g.beta = beta;
    if ((a_kcontig && g.sAkk != 1) || (!a_kcontig && g.sAm != 1) || (b_ncontig && g.sBn != 1) ||
        (!b_ncontig && g.sBkk != 1))
      throw std::invalid_argument("contiguity flags do not match the strides");
    if (prec == TT_F64)
      tt::gemm<double>(g, (const double*)A, (const double*)B, (double*)Cm, a_kcontig, b_ncontig, E.stream);
    else if (prec == TT_F32)
      tt::gemm<float>(g, (const float*)A, (const float*)B, (float*)Cm, a_kcontig, b_ncontig, E.stream);
    else if (prec == TT_BF16)
      tt::gemm_bf16(g, (const uint16_t*)A, (const uint16_t*)B, (float*)Cm, a_kcontig, b_ncontig, E.stream);
    else
      throw std::invalid_argument("unknown precision");
    if (hipStreamSynchronize(E.stream) != hipSuccess) throw tt::HipError("HIP: stream synchronisation failed");
    return TT_OK;
  });
}

int tt_env_update_dev(void* ctx, int side, int rb, int rk, int rb2, int rk2, int RA, int RB, const double* Env,
                      const double* Ubra, const double* Uket, int nnz, const int32_t* A, const int32_t* B,
                      const double* ops, double* out) {
  return guard(ctx, [&](Engine& E) {
    for (int d : {rb, rk, rb2, rk2})
      if (d <= 0 || d % tt::PAD) throw std::invalid_argument("bond dimensions must be positive multiples of 32");
    if (RA <= 0 || RB <= 0) throw std::invalid_argument("channel counts must be positive");
    if (!Env || !Ubra || !Uket || !out || (nnz && (!A || !B || !ops))) throw std::invalid_argument("NULL pointer");
    check_entries(nnz, A, B, RA, RB);
    tt::SiteOp w;
    std::vector<double> o(ops, ops + 16LL * nnz);
    if (side == 0) {
      Engine::build_siteop(w, RB, vec(B, nnz), vec(A, nnz), o, E.stream);
      E.env_left_raw(rb, rk, rb2, rk2, RA, Env, Ubra, Uket, w, RB, out);
    } else if (side == 1) {
      Engine::build_siteop(w, RA, vec(A, nnz), vec(B, nnz), o, E.stream);
      E.env_right_raw(rb, rk, rb2, rk2, RB, Env, Ubra, Uket, w, RA, out);
    } else {
      throw std::invalid_argument("side must be 0 or 1");
    }
    if (hipStreamSynchronize(E.stream) != hipSuccess) throw tt::HipError("HIP: stream synchronisation failed");
    return TT_OK;
  });
}

int tt_heff_energy_grad_dev(void* ctx, int rl, int rr, int RA, int RB, int RC, const double* Lenv, const double* Renv,
                            int nnz1, const int32_t* A1, const int32_t* B1, const double* ops1, int nnz2,
                            const int32_t* A2, const int32_t* B2, const double* ops2, const double* x, double* En,
                            double* gx, double* gL, double* gR, double* gops1, double* gops2) {
  return guard(ctx, [&](Engine& E) {
    if (rl <= 0 || rr <= 0 || rl % tt::PAD || rr % tt::PAD)
      throw std::invalid_argument("rl and rr must be positive multiples of 32");
    if (RA <= 0 || RB <= 0 || RC <= 0) throw std::invalid_argument("channel counts must be positive");
    if (!Lenv || !Renv || !x || !En || !gx || !gL || !gR || !gops1 || !gops2) throw std::invalid_argument("NULL pointer");
    check_entries(nnz1, A1, B1, RA, RB);
    check_entries(nnz2, A2, B2, RB, RC);
    std::vector<int> a1 = vec(A1, nnz1), b1 = vec(B1, nnz1), a2 = vec(A2, nnz2), b2 = vec(B2, nnz2);
    std::vector<double> o1(ops1, ops1 + 16LL * nnz1), o2(ops2, ops2 + 16LL * nnz2);
    std::vector<double> g1, g2;
    E.heff_grad_raw(rl, rr, RA, RB, RC, Lenv, Renv, a1, b1, o1, a2, b2, o2, x, En, gx, gL, gR, g1, g2);
    std::memcpy(gops1, g1.data(), sizeof(double) * g1.size());
    std::memcpy(gops2, g2.data(), sizeof(double) * g2.size());
    return TT_OK;
  });
}

int tt_kernel_timing(void* ctx, int enable, double* stats, int reset) {
  return guard(ctx, [&](Engine& E) {
    if (stats)
      for (int i = 0; i < TT_KT_SLOTS; ++i)
        for (int j = 0; j < 4; ++j) stats[i * 4 + j] = E.kstat[i][j];
    if (reset)
      for (auto& r : E.kstat)
        for (double& v : r) v = 0.0;
    E.kt_on = enable != 0;
    return TT_OK;
  });
}

int tt_energy_mpo_grad(void* ctx, double* En, double* const* gops) {
  return guard(ctx, [&](Engine& E) {
    if (!En || !gops) throw std::invalid_argument("NULL pointer");
    E.mpo_grad(En, gops);
    return TT_OK;
  });
}

}  // extern "C"
