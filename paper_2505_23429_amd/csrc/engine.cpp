// Host orchestration of the additive two-level DMRG hot path on one GPU.
// All tensor arithmetic runs in the kernels of kernels.hip or in rocSOLVER on
// the device; the host only takes decisions on small data (Rayleigh-Ritz
// matrices of the local solver, singular values for truncation, the coarse
// (P+1)x(P+1) pencil).
#include "engine.h"
#include "bsheff.h"

#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <numeric>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>
#include <map>
#include <stdexcept>

namespace tt {

#define HC(x)                                                                                       \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) throw HipError(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)
#define RC(x)                                                                                      \
  do {                                                                                             \
    rocblas_status s_ = (x);                                                                       \
    if (s_ != rocblas_status_success)                                                              \
      throw SolverError(std::string("rocSOLVER/rocBLAS status ") + std::to_string((int)s_) + " at " #x); \
  } while (0)

static const Q2 SITE_Q[4] = {{0, 0}, {1, 1}, {1, -1}, {2, 0}};
static inline Q2 qadd(Q2 a, Q2 b) { return {a[0] + b[0], a[1] + b[1]}; }
static inline Q2 qsub(Q2 a, Q2 b) { return {a[0] - b[0], a[1] - b[1]}; }

static constexpr int QSENT = 1 << 20;  // charge of padding rows/columns: matches no rule

static void upload_q2(DevMem& d, const std::vector<Q2>& v, hipStream_t s) {
  std::vector<int> f(2 * v.size());
  for (size_t i = 0; i < v.size(); ++i) { f[2 * i] = v[i][0]; f[2 * i + 1] = v[i][1]; }
  upload(d, f.data(), f.size() * sizeof(int), s);
}

// charges of a padded label list (sentinel sign: +1 for output-side, -1 for input-side arrays)
static std::vector<Q2> padded_q(const Labels& q, int n, int sent) {
  std::vector<Q2> v(n, Q2{sent * QSENT, 0});
  for (int i = 0; i < (int)q.size() && i < n; ++i) v[i] = q[i];
  return v;
}


// ---------------------------------------------------------------------------
// memory helpers
// ---------------------------------------------------------------------------
// Caching device allocator behind DevMem: released blocks are kept in a
// size-keyed free list and reused, so the many short-lived multi-GB
// environment buffers of a sweep do not go through hipMalloc/hipFree each time.
namespace {
// stream of the worker engine driven by this host thread (null: the main thread)
thread_local hipStream_t tl_stream = nullptr;

class BlockPool {
 public:
  void* get(size_t bytes, size_t& cap) {
    const size_t r = round(bytes);
    {
      std::lock_guard<std::mutex> g(mu_);
      auto it = free_.lower_bound(r);
      if (it != free_.end() && it->first <= r + r / 2) {
        cap = it->first;
        void* p = it->second;
        cached_ -= cap;
        free_.erase(it);
        return p;
      }
    }
    void* p = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    if (hipMalloc(&p, r) != hipSuccess) {
      (void)hipGetLastError();
      trim(0);
      if (hipMalloc(&p, r) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      ++stats_[0];
      stats_[1] += (double)r;
      stats_[2] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    cap = r;
    return p;
  }
  // {device allocations, bytes, seconds in hipMalloc, frees, seconds in hipFree}
  std::array<double, 5> stats() {
    std::lock_guard<std::mutex> g(mu_);
    return stats_;
  }
  void put(void* p, size_t cap) {
    const size_t limit = max_cached();
    // work queued on the releasing thread's stream may still read the block (a
    // worker thread's blocks are used on its own stream only; other threads wait
    // for the whole device)
    if (tl_stream) (void)hipStreamSynchronize(tl_stream);
    else (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> g(mu_);
    free_.emplace(cap, p);
    cached_ += cap;
    if (cached_ > limit) trim_locked(limit / 2);
  }
  void trim(size_t target) {
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> g(mu_);
    trim_locked(target);
  }

 private:
  // released blocks are kept up to 60% of the device memory (a failed allocation
  // empties the cache and retries)
  static size_t max_cached() {
    static const size_t lim = [] {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess || tot == 0) {
        (void)hipGetLastError();
        return size_t(48) << 30;
      }
      return tot / 10 * 6;
    }();
    return lim;
  }
  // size classes: powers of two up to 1 MiB, then steps of about 1/8 (2 MiB minimum), so
  // that the many slightly different sizes of a sweep's environments share blocks
  static size_t round(size_t b) {
    if (b <= (size_t(1) << 20)) {
      size_t r = 256;
      while (r < b) r <<= 1;
      return r;
    }
    const size_t g = size_t(2) << 20;
    size_t r = g;
    while (r < b) r += std::max(g, (r / 8) / g * g);
    return r;
  }
  void trim_locked(size_t target) {
    while (cached_ > target && !free_.empty()) {
      auto it = std::prev(free_.end());
      const auto t0 = std::chrono::steady_clock::now();
      (void)hipFree(it->second);
      stats_[3] += 1.0;
      stats_[4] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      cached_ -= it->first;
      free_.erase(it);
    }
  }
  std::array<double, 5> stats_ = {};
  std::mutex mu_;
  std::multimap<size_t, void*> free_;
  size_t cached_ = 0;
};
BlockPool& pool() {
  static BlockPool* p = new BlockPool;  // lives until process exit
  return *p;
}

// Large blocks (the environments and intermediates of a sweep, up to ~10 GB at
// chi = 1024) come from chunks of device memory that are carved best-fit and
// coalesced on release, so that requests of ever-changing sizes do not each cost
// a hipMalloc.  A chunk goes back to the device only when a new chunk cannot be
// obtained and the chunk is entirely free.
class Arena {
 public:
  static constexpr size_t kMin = size_t(64) << 20;  // requests from this size on
  void* get(size_t bytes, size_t& cap) {
    const size_t r = (bytes + kAlign - 1) / kAlign * kAlign;
    std::lock_guard<std::mutex> g(mu_);
    for (int attempt = 0; attempt < 3; ++attempt) {
      auto it = by_size_.lower_bound(r);
      if (it != by_size_.end()) {
        char* p = it->second;
        const size_t sz = it->first;
        by_size_.erase(it);
        by_addr_.erase(p);
        if (sz > r) insert_free(p + r, sz - r);
        used_[p] = r;
        cap = r;
        return p;
      }
      if (attempt == 0 && grow(std::max(r, kChunk))) continue;
      if (attempt <= 1) {
        release_free_chunks();
        if (grow(r)) continue;
      }
    }
    return nullptr;
  }
  bool owns(void* p) {
    std::lock_guard<std::mutex> g(mu_);
    return used_.count((char*)p) != 0;
  }
  void put(void* p) {
    if (tl_stream) (void)hipStreamSynchronize(tl_stream);
    else (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> g(mu_);
    auto it = used_.find((char*)p);
    if (it == used_.end()) return;
    const size_t sz = it->second;
    used_.erase(it);
    insert_free((char*)p, sz);
  }
  std::array<double, 3> stats() {
    std::lock_guard<std::mutex> g(mu_);
    return {(double)chunks_.size(), (double)total_, grow_s_};
  }

 private:
  static constexpr size_t kAlign = size_t(2) << 20;
  static constexpr size_t kChunk = size_t(32) << 30;
  bool grow(size_t size) {
    void* p = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    if (hipMalloc(&p, size) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    grow_s_ += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    chunks_[(char*)p] = size;
    total_ += size;
    insert_free((char*)p, size);
    return true;
  }
  char* chunk_of(char* p) const {
    auto it = chunks_.upper_bound(p);
    return it == chunks_.begin() ? nullptr : std::prev(it)->first;
  }
  void insert_free(char* p, size_t sz) {
    char* c = chunk_of(p);
    // merge with the following free segment of the same chunk
    auto nx = by_addr_.find(p + sz);
    if (nx != by_addr_.end() && chunk_of(nx->first) == c) {
      erase_size(nx->first, nx->second);
      sz += nx->second;
      by_addr_.erase(nx);
    }
    // and with the preceding one
    auto pv = by_addr_.lower_bound(p);
    if (pv != by_addr_.begin()) {
      --pv;
      if (pv->first + pv->second == p && chunk_of(pv->first) == c) {
        erase_size(pv->first, pv->second);
        p = pv->first;
        sz += pv->second;
        by_addr_.erase(pv);
      }
    }
    by_addr_[p] = sz;
    by_size_.emplace(sz, p);
  }
  void erase_size(char* p, size_t sz) {
    auto range = by_size_.equal_range(sz);
    for (auto it = range.first; it != range.second; ++it)
      if (it->second == p) {
        by_size_.erase(it);
        return;
      }
  }
  void release_free_chunks() {
    (void)hipDeviceSynchronize();
    for (auto it = chunks_.begin(); it != chunks_.end();) {
      auto f = by_addr_.find(it->first);
      if (f != by_addr_.end() && f->second == it->second) {
        erase_size(f->first, f->second);
        by_addr_.erase(f);
        (void)hipFree(it->first);
        total_ -= it->second;
        it = chunks_.erase(it);
      } else {
        ++it;
      }
    }
  }
  std::mutex mu_;
  std::map<char*, size_t> chunks_, by_addr_, used_;
  std::multimap<size_t, char*> by_size_;
  size_t total_ = 0;
  double grow_s_ = 0.0;
};
Arena& arena() {
  static Arena* a = new Arena;  // lives until process exit
  return *a;
}
}  // namespace

static thread_local const ExtAlloc* tl_ext = nullptr;
static thread_local hipStream_t tl_ext_stream = nullptr;
void set_thread_allocator(const ExtAlloc* a, hipStream_t s) {
  tl_ext = (a && a->alloc) ? a : nullptr;
  tl_ext_stream = s;
}

void DevMem::release() {
  if (p && own) {
    if (ext) {
      // work queued on the releasing thread's stream may still read the block
      if (tl_stream) (void)hipStreamSynchronize(tl_stream);
      else (void)hipDeviceSynchronize();
      ext->free(p, (void*)ext_stream, ext->user);
    } else if (cap >= Arena::kMin && arena().owns(p)) {
      arena().put(p);
    } else {
      pool().put(p, cap);
    }
  }
  p = nullptr;
  n = 0;
  cap = 0;
  own = true;
  ext = nullptr;
  ext_stream = nullptr;
}
// allocation budget of the task running on this thread (worker_alloc_limit; -1: none)
static thread_local long long tl_alloc_budget = -1;
static void charge_budget(size_t bytes) {
  if (tl_alloc_budget < 0) return;
  if ((long long)bytes > tl_alloc_budget)
    throw DeviceOOM("device allocation of " + std::to_string(bytes) + " bytes failed (task allocation limit)");
  tl_alloc_budget -= (long long)bytes;
}

// a new block of at least `bytes` for m (released first): the caller's allocator of
// this thread's call when there is one, else the arena (large) or the block pool
static void acquire(DevMem& m, size_t bytes) {
  charge_budget(bytes);
  if (tl_ext) {
    m.p = tl_ext->alloc(bytes, (void*)tl_ext_stream, tl_ext->user);
    m.cap = m.p ? bytes : 0;
    m.ext = m.p ? tl_ext : nullptr;
    m.ext_stream = m.p ? tl_ext_stream : nullptr;
  } else {
    m.p = bytes >= Arena::kMin ? arena().get(bytes, m.cap) : nullptr;
    if (!m.p) m.p = pool().get(bytes, m.cap);
  }
  if (!m.p) {
    m.cap = 0;
    throw DeviceOOM("device allocation of " + std::to_string(bytes) + " bytes failed");
  }
}

void DevMem::ensure(size_t bytes) {
  if (own && p && bytes <= cap) {
    if (bytes > n) n = bytes;
    return;
  }
  if (bytes <= n) return;
  release();
  if (bytes == 0) return;
  acquire(*this, bytes);
  n = bytes;
}
void DevMem::resize_zero(size_t bytes, hipStream_t s) {
  if (!(own && p && bytes <= cap)) {
    release();
    if (bytes) acquire(*this, bytes);
  }
  n = bytes;
  if (bytes) fill(p, bytes, s);
}
void upload(DevMem& m, const void* h, size_t bytes, hipStream_t s) {
  m.ensure(bytes);
  if (bytes) HC(hipMemcpyAsync(m.p, h, bytes, hipMemcpyHostToDevice, s));
  HC(hipStreamSynchronize(s));
}
void download(void* h, const DevMem& m, size_t bytes, hipStream_t s) {
  if (bytes) HC(hipMemcpyAsync(h, m.p, bytes, hipMemcpyDeviceToHost, s));
  HC(hipStreamSynchronize(s));
}
static void d2h(void* h, const void* d, size_t bytes, hipStream_t s) {
  if (bytes) HC(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
  HC(hipStreamSynchronize(s));
}
static DevMem upload_ints(const std::vector<int>& v, hipStream_t s) {
  DevMem m;
  upload(m, v.data(), v.size() * sizeof(int), s);
  return m;
}
static DevMem upload_dbl(const std::vector<double>& v, hipStream_t s) {
  DevMem m;
  upload(m, v.data(), v.size() * sizeof(double), s);
  return m;
}

// ---------------------------------------------------------------------------
// small dense symmetric eigensolver (cyclic Jacobi), host FP64
// ---------------------------------------------------------------------------
static void jacobi_eig(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        if (i != j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
      }
    if (off <= 1e-30 * std::max(tot, 1e-300)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  // sort ascending
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[(size_t)a * n + a] < A[(size_t)b * n + b]; });
  w.resize(n);
  std::vector<double> V2((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    w[j] = A[(size_t)idx[j] * n + idx[j]];
    for (int k = 0; k < n; ++k) V2[(size_t)k * n + j] = V[(size_t)k * n + idx[j]];
  }
  V.swap(V2);
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------
Engine::Engine(const tt_opts& o)
    : opts(o), prob(std::make_shared<Problem>()), L(prob->L), mpo(prob->mpo), Rb(prob->Rb), chan_q(prob->chan_q),
      chan_q_dev(prob->chan_q_dev) {
  const char* v = std::getenv("TT_VERBOSE");
  verbose_level = v ? std::atoi(v) : 0;
  verbose = verbose_level > 0;
  HC(hipSetDevice(o.device));
  ext.alloc = o.dev_alloc;
  ext.free = o.dev_free;
  ext.user = o.alloc_user;
  if (o.stream) {
    stream = (hipStream_t)o.stream;
    own_stream = false;
  } else {
    HC(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  }
  RC(rocblas_create_handle(&blas));
  RC(rocblas_set_stream(blas, stream));
  HC(hipEventCreate(&ev0));
  HC(hipEventCreate(&ev1));
  noalloc = noalloc_scratch(o.device);  // this device is current (set above)
}
Engine::Engine(const Engine& parent, int)
    : opts(parent.opts), prob(parent.prob), L(prob->L), mpo(prob->mpo), Rb(prob->Rb), chan_q(prob->chan_q),
      chan_q_dev(prob->chan_q_dev) {
  verbose = parent.verbose;
  verbose_level = parent.verbose_level;
  have_mpo = parent.have_mpo;
  ext = parent.ext;
  HC(hipSetDevice(opts.device));
  HC(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  RC(rocblas_create_handle(&blas));
  RC(rocblas_set_stream(blas, stream));
  HC(hipEventCreate(&ev0));
  HC(hipEventCreate(&ev1));
}
Engine::~Engine() {
  if (stream) (void)hipStreamSynchronize(stream);
  workers.clear();
  if (blas) rocblas_destroy_handle(blas);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  for (hipEvent_t& ev : kt_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (stream && own_stream) (void)hipStreamDestroy(stream);
}

void Engine::release_workspaces() {
  for (DevMem* m : {&ws0, &ws1, &ws2, &ws3, &wsd, &wsp, &dav_V, &dav_AV, &dav_t, &dav_u, &dav_Au, &dav_c, &dav_mask, &dav_xd, &dav_yd, &dav_dc, &dav_uk, &dav_tk,
                    &dav_t2, &dav_t3, &wlow_x, &wlow_y, &wlow_L, &wlow_R, &wlow_Rt, &envq_o, &envq_i, &bs_t1, &bs_t2,
                    &bs_t3, &bs_part, &bs_tmp, &be_t1, &be_panel, &be_up, &be_tmp})
    m->release();
  for (int b = 0; b < 4; ++b) {
    bs_gg1[b].release();
    bs_gg2[b].release();
  }
  bs_zero_serial = -1;
  bs_zero_prec = -1;
  bs_gg_serial = -1;
  bs_gg_prec = -1;
  for (auto& q : bs_gg_ptr) q = nullptr;
}

void Engine::free_caches() {
  Vc.clear();
  Wc.clear();
  Lenv.clear();
  Renv.clear();
  FL.clear();
  FR.clear();
  subs.clear();
  have_local = false;
}

void siteop_csr(int nout, const std::vector<int>& out_idx, const std::vector<int>& in_idx,
                const std::vector<double>& ops, std::vector<int>& ptr, std::vector<int>& src,
                std::vector<double>& op64, std::vector<float>& op32) {
  const int nnz = (int)out_idx.size();
  std::vector<int> order(nnz);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return out_idx[a] < out_idx[b]; });
  ptr.assign(nout + 1, 0);
  src.assign(std::max(nnz, 1), 0);
  op64.assign((size_t)std::max(nnz, 1) * 16, 0.0);
  op32.assign((size_t)std::max(nnz, 1) * 16, 0.f);
  for (int e = 0; e < nnz; ++e) {
    if (out_idx[e] < 0 || out_idx[e] >= nout) throw std::runtime_error("MPO entry channel out of range");
    ptr[out_idx[e] + 1]++;
  }
  for (int c = 0; c < nout; ++c) ptr[c + 1] += ptr[c];
  for (int k = 0; k < nnz; ++k) {
    int e = order[k];
    src[k] = in_idx[e];
    for (int j = 0; j < 16; ++j) {
      op64[(size_t)k * 16 + j] = ops[(size_t)e * 16 + j];
      op32[(size_t)k * 16 + j] = (float)ops[(size_t)e * 16 + j];
    }
  }
}

void Engine::build_siteop(SiteOp& so, int nout, const std::vector<int>& out_idx, const std::vector<int>& in_idx,
                          const std::vector<double>& ops, hipStream_t s) {
  const int nnz = (int)out_idx.size();
  std::vector<int> ptr, src;
  std::vector<double> op64;
  std::vector<float> op32;
  siteop_csr(nout, out_idx, in_idx, ops, ptr, src, op64, op32);
  so.nout = nout;
  so.nnz = nnz;
  so.hptr = ptr;
  so.hsrc.assign(src.begin(), src.begin() + nnz);
  so.hop.assign(op64.begin(), op64.begin() + (size_t)nnz * 16);
  upload(so.ptr, ptr.data(), ptr.size() * sizeof(int), s);
  upload(so.src, src.data(), src.size() * sizeof(int), s);
  upload(so.op64, op64.data(), op64.size() * sizeof(double), s);
  upload(so.op32, op32.data(), op32.size() * sizeof(float), s);
}

void Engine::set_mpo(int L_, const int* R, const int* nnz, const int32_t* const* A, const int32_t* const* B,
                     const double* const* ops, const int32_t* const* cq, const int* block) {
  if (L_ < 2) throw std::invalid_argument("L must be >= 2");
  if (R[0] != 1 || R[L_] != 1) throw std::invalid_argument("MPO boundary bond dimensions must be 1");
  for (int k = 0; k <= L_; ++k)
    if (R[k] <= 0) throw std::invalid_argument("MPO bond dimension must be positive");
  std::vector<SiteMPO> m(L_);
  std::vector<Labels> q(L_ + 1);
  for (int k = 0; k <= L_; ++k) {
    q[k].resize(R[k]);
    for (int c = 0; c < R[k]; ++c) q[k][c] = {cq[k][2 * c], cq[k][2 * c + 1]};
  }
  for (int k = 0; k < L_; ++k) {
    SiteMPO& s = m[k];
    s.Rl = R[k];
    s.Rr = R[k + 1];
    s.A.assign(A[k], A[k] + nnz[k]);
    s.B.assign(B[k], B[k] + nnz[k]);
    s.ops.assign(ops[k], ops[k] + (size_t)nnz[k] * 16);
    for (int e = 0; e < nnz[k]; ++e) {
      if (s.A[e] < 0 || s.A[e] >= s.Rl || s.B[e] < 0 || s.B[e] >= s.Rr)
        throw std::invalid_argument("MPO entry index out of range at site " + std::to_string(k));
      // charge conservation: q(A) + q(s') - q(s) == q(B) for every nonzero op element
      for (int sp = 0; sp < 4; ++sp)
        for (int sn = 0; sn < 4; ++sn)
          if (s.ops[(size_t)e * 16 + sp * 4 + sn] != 0.0) {
            Q2 lhs = qsub(qadd(q[k][s.A[e]], SITE_Q[sp]), SITE_Q[sn]);
            if (lhs != q[k + 1][s.B[e]])
              throw std::invalid_argument("MPO entry violates channel charges at site " + std::to_string(k));
          }
    }
    int p0 = block ? block[4 * k] : -1, p1 = block ? block[4 * k + 1] : -1;
    int q0 = block ? block[4 * k + 2] : -1, q1 = block ? block[4 * k + 3] : -1;
    std::vector<int> rA, rB, nA, nB, vA, vB, xA, xB;
    std::vector<double> rO, nO, vO, xO;
    if (p0 >= 0 && p1 > p0 && q0 >= 0 && q1 > q0) {
      if (p1 > s.Rl || q1 > s.Rr) throw std::invalid_argument("coefficient block out of range");
      s.has_block = true;
      s.p0 = p0; s.p1 = p1; s.q0 = q0; s.q1 = q1;
      const int nP = p1 - p0, nQ = q1 - q0;
      std::vector<double> Vh((size_t)nQ * nP, 0.0);
      for (int e = 0; e < nnz[k]; ++e) {
        const double* o = &s.ops[(size_t)e * 16];
        bool in_blk = s.A[e] >= p0 && s.A[e] < p1 && s.B[e] >= q0 && s.B[e] < q1;
        if (in_blk) {
          double c = o[0];
          for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j)
              if (std::fabs(o[i * 4 + j] - (i == j ? c : 0.0)) > 1e-15 * std::max(1.0, std::fabs(c)))
                throw std::invalid_argument("coefficient block entry without identity local operator");
          Vh[(size_t)(s.B[e] - q0) * nP + (s.A[e] - p0)] += c;
        } else {
          nA.push_back(s.A[e]); nB.push_back(s.B[e]);
          nO.insert(nO.end(), o, o + 16);
        }
      }
      upload(s.V, Vh.data(), Vh.size() * sizeof(double), stream);
      // charge classes of the block (a coupling of unequal channel charges would break
      // charge conservation: the block entries carry the identity local operator)
      {
        std::map<Q2, int> cid;
        for (int pp = 0; pp < nP; ++pp) {
          const Q2 d = q[k][p0 + pp];
          auto it = cid.find(d);
          if (it == cid.end()) {
            it = cid.emplace(d, (int)s.vcls.size()).first;
            s.vcls.emplace_back();
            s.vcls.back().d = d;
          }
          s.vcls[it->second].P.push_back(pp);
        }
        for (int qq = 0; qq < nQ; ++qq) {
          auto it = cid.find(q[k + 1][q0 + qq]);
          if (it != cid.end()) s.vcls[it->second].Q.push_back(qq);
        }
        for (int qq = 0; qq < nQ; ++qq)
          for (int pp = 0; pp < nP; ++pp)
            if (Vh[(size_t)qq * nP + pp] != 0.0 && q[k + 1][q0 + qq] != q[k][p0 + pp])
              throw std::invalid_argument("coefficient block couples channels of different charge at site " +
                                          std::to_string(k));
        for (auto& c : s.vcls) {
          std::vector<double> vc(std::max<size_t>(c.Q.size() * c.P.size(), 1), 0.0);
          for (size_t i = 0; i < c.Q.size(); ++i)
            for (size_t j = 0; j < c.P.size(); ++j) vc[i * c.P.size() + j] = Vh[(size_t)c.Q[i] * nP + c.P[j]];
          c.Pd = upload_ints(c.P, stream);
          c.Qd = upload_ints(c.Q.empty() ? std::vector<int>{0} : c.Q, stream);
          upload(c.V, vc.data(), vc.size() * sizeof(double), stream);
        }
      }
      static const double Id[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
      // left use: output q gathers from virtual input Rl + (q - q0)
      vA = nA; vB = nB; vO = nO;
      for (int qq = q0; qq < q1; ++qq) {
        vA.push_back(s.Rl + (qq - q0)); vB.push_back(qq);
        vO.insert(vO.end(), Id, Id + 16);
      }
      build_siteop(s.byB_left, s.Rr, vB, vA, vO, stream);
      build_siteop(s.byB_noblk, s.Rr, nB, nA, nO, stream);
      // right use: output p (left bond) gathers from virtual input Rr + (p - p0)
      xA = nA; xB = nB; xO = nO;
      for (int pp = p0; pp < p1; ++pp) {
        xA.push_back(pp); xB.push_back(s.Rr + (pp - p0));
        xO.insert(xO.end(), Id, Id + 16);
      }
      build_siteop(s.byA_right, s.Rl, xA, xB, xO, stream);
      // second site of a window: block row p feeds the virtual output Rr + (p - p0)
      std::vector<int> yA = nA, yB = nB;
      std::vector<double> yO = nO;
      for (int pp = p0; pp < p1; ++pp) {
        yA.push_back(pp); yB.push_back(s.Rr + (pp - p0));
        yO.insert(yO.end(), Id, Id + 16);
      }
      build_siteop(s.byB_rightv, s.Rr + nP, yB, yA, yO, stream);
    }
    build_siteop(s.byB, s.Rr, s.B, s.A, s.ops, stream);
    build_siteop(s.byA, s.Rl, s.A, s.B, s.ops, stream);
  }
  chan_q_dev.clear();
  chan_q_dev.resize(L_ + 1);
  for (int k = 0; k <= L_; ++k) {
    std::vector<int> flat;
    for (auto& x : q[k]) { flat.push_back(x[0]); flat.push_back(x[1]); }
    upload(chan_q_dev[k], flat.data(), flat.size() * sizeof(int), stream);
  }
  mpo = std::move(m);
  chan_q = std::move(q);
  Rb.assign(R, R + L_ + 1);
  if (have_mps && L != L_) have_mps = false;
  L = L_;
  have_mpo = true;
  free_caches();
}

// ---------------------------------------------------------------------------
// per-kernel timing of the effective-Hamiltonian product (HIP events on the
// library stream; enabled by tt_kernel_timing)
// ---------------------------------------------------------------------------
double Engine::now() {
  HC(hipStreamSynchronize(stream));
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

namespace {
// accumulates wall time (stream synchronised) of a scope in verbose mode
struct ScopeTimer {
  Engine& E;
  double& acc;
  int& cnt;
  double t0 = 0.0;
  ScopeTimer(Engine& e, double& a, int& c) : E(e), acc(a), cnt(c) {
    if (E.verbose) t0 = E.now();
  }
  ~ScopeTimer() {
    if (!E.verbose) return;
    try {
      acc += E.now() - t0;
      ++cnt;
    } catch (...) {
    }
  }
};
}  // namespace

void Engine::kt_begin() {
  if (!kt_on) return;
  if (!kt_ev[0]) HC(hipEventCreate(&kt_ev[0]));
  HC(hipEventRecord(kt_ev[0], stream));
  kt_n = 1;
}
void Engine::kt_mark(int slot) {
  if (!kt_on || kt_n <= 0 || kt_n > KT_SLOTS) return;
  if (!kt_ev[kt_n]) HC(hipEventCreate(&kt_ev[kt_n]));
  HC(hipEventRecord(kt_ev[kt_n], stream));
  kt_slot[kt_n] = slot;
  ++kt_n;
}
void Engine::kt_end(const double* fl, const double* by) {
  if (!kt_on || kt_n <= 1) return;
  HC(hipEventSynchronize(kt_ev[kt_n - 1]));
  bool seen[KT_SLOTS] = {};
  for (int i = 1; i < kt_n; ++i) {
    float ms = 0.f;
    HC(hipEventElapsedTime(&ms, kt_ev[i - 1], kt_ev[i]));
    const int sl = kt_slot[i];
    kstat[sl][0] += ms;
    seen[sl] = true;
  }
  for (int sl = 0; sl < KT_SLOTS; ++sl)
    if (seen[sl]) {
      kstat[sl][1] += 1.0;
      kstat[sl][2] += fl[sl];
      kstat[sl][3] += by[sl];
    }
  kt_n = 0;
}

// dense-bond work of the dense product (all channels, true sizes)
static void dense_work(const Engine& E, int elem, int RB, double* fl, double* by) {
  const double rl = E.cur_rl, rr = E.cur_rr, slab = rl * 16.0 * rr;
  for (int i = 0; i < Engine::KT_SLOTS; ++i) fl[i] = by[i] = 0.0;
  fl[0] = 2.0 * E.cur_RA * rl * rl * 16.0 * rr;
  fl[7] = 2.0 * 16.0 * rl * rr * rr * E.cur_RC;
  by[1] = (double)elem * slab * (E.cur_RA + RB);
  by[4] = (double)elem * slab * (RB + E.cur_RC);
}

// ---------------------------------------------------------------------------
// effective Hamiltonian product (K1)
//   T1[A][a'][s1 s2 b] = L_A x               batched MFMA GEMM
//   T2[B][a'][s1'][s2 b] = W1 mix over s1    sparse, memory bound
//   T3[C][a' s1'][s2'][b] = W2 mix over s2
//   y[(a' s1' s2')][b'] = sum_C T3[C] R_C^T  MFMA GEMM with K = (C, b)
// ---------------------------------------------------------------------------
template <class T>
static const T* siteop_ops(const SiteOp& so);
template <>
const double* siteop_ops<double>(const SiteOp& so) { return so.op64.as<double>(); }
template <>
const float* siteop_ops<float>(const SiteOp& so) { return so.op32.as<float>(); }

// The dense two-site product on raw tables and workspaces:
//   T1 = L_A x (batched GEMM over the channels A), T2 = W1 mix of T1, T3 = W2 mix of T2
//   (in T1's space), y = sum_C T3_C R_C^T (+ the second-site coefficient block's channels).
// Site k's entries are given grouped by output channel (ptr[nout + 1], src[nnz], ops[nnz][16]).
// ws_a holds max(RA, RC) slabs of rl*16*rr elements, ws_b holds RB slabs.  With timed, the
// kernels are timed into the engine's per-kernel statistics.
template <class T>
void heff_dense(Engine& E, int rl, int rr, int RA, const T* Lv, int RB, const int* p1, const int* s1, const T* o1,
                int RC, const int* p2, const int* s2, const T* o2, const T* Rv, const T* x, T* y, T* ws_a, T* ws_b,
                const T* Rtil, int P0, int nP, const WinTabs* tabs, bool timed) {
  const long long slab = (long long)rl * 16 * rr;
  T* T1 = ws_a;
  T* T2 = ws_b;
  GemmArgs g{};
  g.M = rl; g.N = 16 * rr; g.K = rl; g.batch = RA; g.kin = rl;
  g.sAb = (long long)rl * rl; g.sAm = rl; g.sAkb = 0; g.sAkk = 1;
  g.sBb = 0; g.sBkb = 0; g.sBkk = 16LL * rr; g.sBn = 1;
  g.sCb = slab; g.sCm = 16LL * rr; g.alpha = 1.0; g.beta = 0.0;
  MixQ q1, q2;
  if (tabs) {
    g.kmode = 1; g.mtiles = tabs->m1tiles; g.ntiles = tabs->n1tiles;
    g.ktab = tabs->k1tab.as<int>(); g.skip = tabs->k1skip.as<unsigned char>();
    q1.qo = tabs->qo1.as<int2>(); q1.qi = tabs->qi1.as<int2>(); q1.qc = tabs->qcB;
    q2.qo = tabs->qo2.as<int2>(); q2.qi = tabs->qi2.as<int2>(); q2.qc = tabs->qcC;
  }
  if (timed) E.kt_begin();
  gemm<T>(g, Lv, x, T1, true, true, E.stream);
  if (timed) E.kt_mark(0);
  mix<T>(RB, p1, s1, o1, T1, slab, T2, slab, rl, 4 * rr, E.stream, tabs ? &q1 : nullptr);
  if (timed) E.kt_mark(1);
  T* T3 = ws_a;
  mix<T>(RC, p2, s2, o2, T2, slab, T3, slab, 4 * rl, rr, E.stream, tabs ? &q2 : nullptr);
  if (timed) E.kt_mark(4);
  GemmArgs h{};
  h.M = 16 * rl; h.N = rr; h.K = RC * rr; h.batch = 1; h.kin = rr;
  h.sAb = 0; h.sAm = rr; h.sAkb = slab; h.sAkk = 1;
  h.sBb = 0; h.sBkb = (long long)rr * rr; h.sBkk = 1; h.sBn = rr;
  h.sCb = 0; h.sCm = rr; h.alpha = 1.0; h.beta = 0.0;
  if (tabs) {
    h.kmode = 2; h.nkb = RC; h.ntiles = tabs->n4tiles; h.ktab = tabs->k4tab.as<int>();
  }
  gemm<T>(h, T3, Rv, y, true, false, E.stream);
  if (Rtil && nP > 0) {
    h.K = nP * rr;
    h.beta = 1.0;
    if (tabs) { h.nkb = nP; h.ktab = tabs->k4tabP.as<int>(); }
    gemm<T>(h, T2 + (long long)P0 * slab, Rtil, y, true, false, E.stream);
  }
  if (timed) {
    E.kt_mark(7);
    double fl[Engine::KT_SLOTS], by[Engine::KT_SLOTS];
    dense_work(E, sizeof(T), RB, fl, by);
    E.kt_end(fl, by);
  }
}
template void heff_dense<double>(Engine&, int, int, int, const double*, int, const int*, const int*, const double*,
                                 int, const int*, const int*, const double*, const double*, const double*, double*,
                                 double*, double*, const double*, int, int, const WinTabs*, bool);
template void heff_dense<float>(Engine&, int, int, int, const float*, int, const int*, const int*, const float*, int,
                                const int*, const int*, const float*, const float*, const float*, float*, float*,
                                float*, const float*, int, int, const WinTabs*, bool);

template <class T>
void Engine::heff(int rl, int rr, int RA, const T* Lv, const SiteOp& w1, int RB, const SiteOp& w2, int RC,
                  const T* Rv, const T* x, T* y, const T* Rtil, int P0, int nP, const WinTabs* tabs) {
  const long long slab = (long long)rl * 16 * rr;
  ws0.ensure(sizeof(T) * slab * std::max(RA, RC));
  ws1.ensure(sizeof(T) * slab * RB);
  if (w1.nout != RB || w2.nout != RC) throw std::runtime_error("heff: channel count mismatch");
  heff_dense<T>(*this, rl, rr, RA, Lv, RB, w1.ptr.as<int>(), w1.src.as<int>(), siteop_ops<T>(w1), RC,
                w2.ptr.as<int>(), w2.src.as<int>(), siteop_ops<T>(w2), Rv, x, y, ws0.as<T>(), ws1.as<T>(), Rtil, P0,
                nP, tabs, true);
}
template void Engine::heff<double>(int, int, int, const double*, const SiteOp&, int, const SiteOp&, int, const double*,
                                   const double*, double*, const double*, int, int, const WinTabs*);
template void Engine::heff<float>(int, int, int, const float*, const SiteOp&, int, const SiteOp&, int, const float*,
                                  const float*, float*, const float*, int, int, const WinTabs*);

// BF16 operands, FP32 accumulation and FP32 intermediates.  The second mix writes
// FP32; T3 is rounded to BF16 for the last GEMM.
__global__ void round_bf16_kernel(const float* a, uint16_t* b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    uint32_t u = __float_as_uint(a[i]);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    b[i] = (uint16_t)(u >> 16);
  }
}
static void round_bf16(const float* a, uint16_t* b, size_t n, hipStream_t s) {
  if (!n) return;
  unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 1u << 20);
  hipLaunchKernelGGL(round_bf16_kernel, dim3(nb), dim3(256), 0, s, a, b, n);
  HC(hipGetLastError());
}

void Engine::heff_bf16(int rl, int rr, int RA, const uint16_t* Lv, const SiteOp& w1, int RB, const SiteOp& w2, int RC,
                       const uint16_t* Rv, const uint16_t* x, float* y, const uint16_t* Rtil, int P0, int nP,
                       const WinTabs* tabs) {
  const long long slab = (long long)rl * 16 * rr;
  ws0.ensure(sizeof(float) * slab * std::max(RA, RC));
  ws1.ensure(sizeof(float) * slab * RB);
  float* T1 = ws0.as<float>();
  float* T2 = ws1.as<float>();
  GemmArgs g{};
  g.M = rl; g.N = 16 * rr; g.K = rl; g.batch = RA; g.kin = rl;
  g.sAb = (long long)rl * rl; g.sAm = rl; g.sAkb = 0; g.sAkk = 1;
  g.sBb = 0; g.sBkb = 0; g.sBkk = 16LL * rr; g.sBn = 1;
  g.sCb = slab; g.sCm = 16LL * rr; g.alpha = 1.0; g.beta = 0.0;
  MixQ q1, q2;
  if (tabs) {
    g.kmode = 1; g.mtiles = tabs->m1tiles; g.ntiles = tabs->n1tiles;
    g.ktab = tabs->k1tab.as<int>(); g.skip = tabs->k1skip.as<unsigned char>();
    q1.qo = tabs->qo1.as<int2>(); q1.qi = tabs->qi1.as<int2>(); q1.qc = tabs->qcB;
    q2.qo = tabs->qo2.as<int2>(); q2.qi = tabs->qi2.as<int2>(); q2.qc = tabs->qcC;
  }
  kt_begin();
  gemm_bf16(g, Lv, x, T1, true, true, stream);
  kt_mark(0);
  mix<float>(w1.nout, w1.ptr.as<int>(), w1.src.as<int>(), w1.op32.as<float>(), T1, slab, T2, slab, rl, 4 * rr, stream,
             tabs ? &q1 : nullptr);
  kt_mark(1);
  float* T3 = ws0.as<float>();
  mix<float>(w2.nout, w2.ptr.as<int>(), w2.src.as<int>(), w2.op32.as<float>(), T2, slab, T3, slab, 4 * rl, rr, stream,
             tabs ? &q2 : nullptr);
  kt_mark(4);
  ws2.ensure(sizeof(uint16_t) * slab * std::max(RC, nP));
  uint16_t* T3b = ws2.as<uint16_t>();
  round_bf16(T3, T3b, (size_t)slab * RC, stream);
  GemmArgs h{};
  h.M = 16 * rl; h.N = rr; h.K = RC * rr; h.batch = 1; h.kin = rr;
  h.sAb = 0; h.sAm = rr; h.sAkb = slab; h.sAkk = 1;
  h.sBb = 0; h.sBkb = (long long)rr * rr; h.sBkk = 1; h.sBn = rr;
  h.sCb = 0; h.sCm = rr; h.alpha = 1.0; h.beta = 0.0;
  if (tabs) {
    h.kmode = 2; h.nkb = RC; h.ntiles = tabs->n4tiles; h.ktab = tabs->k4tab.as<int>();
  }
  gemm_bf16(h, T3b, Rv, y, true, false, stream);
  if (Rtil && nP > 0) {
    round_bf16(T2 + (long long)P0 * slab, T3b, (size_t)slab * nP, stream);
    h.K = nP * rr;
    h.beta = 1.0;
    if (tabs) { h.nkb = nP; h.ktab = tabs->k4tabP.as<int>(); }
    gemm_bf16(h, T3b, Rtil, y, true, false, stream);
  }
  kt_mark(7);
  {
    double fl[KT_SLOTS], by[KT_SLOTS];
    dense_work(*this, 4, RB, fl, by);
    kt_end(fl, by);
  }
}

// ---------------------------------------------------------------------------
// environment updates (K2 / K3), FP64, padded dims
// ---------------------------------------------------------------------------
void Engine::env_left_raw(int rb, int rk, int rb2, int rk2, int RA, const double* E, const double* Ubra,
                          const double* Uket, const SiteOp& w, int RB, double* out, const MixQ* q) {
  const long long sl = (long long)rb * 4 * rk2;
  ws2.ensure(sizeof(double) * sl * RA);
  ws3.ensure(sizeof(double) * sl * RB);
  double* T = ws2.as<double>();
  double* Tp = ws3.as<double>();
  GemmArgs g{};
  g.M = rb; g.N = 4 * rk2; g.K = rk; g.batch = RA; g.kin = rk;
  g.sAb = (long long)rb * rk; g.sAm = rk; g.sAkb = 0; g.sAkk = 1;
  g.sBb = 0; g.sBkb = 0; g.sBkk = 4LL * rk2; g.sBn = 1;
  g.sCb = sl; g.sCm = 4LL * rk2; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, E, Uket, T, true, true, stream);
  mix<double>(w.nout, w.ptr.as<int>(), w.src.as<int>(), w.op64.as<double>(), T, sl, Tp, sl, rb, rk2, stream, q);
  GemmArgs h{};
  h.M = rb2; h.N = rk2; h.K = 4 * rb; h.batch = RB; h.kin = 4 * rb;
  h.sAb = 0; h.sAm = 1; h.sAkb = 0; h.sAkk = rb2;
  h.sBb = sl; h.sBkb = 0; h.sBkk = rk2; h.sBn = 1;
  h.sCb = (long long)rb2 * rk2; h.sCm = rk2; h.alpha = 1.0; h.beta = 0.0;
  gemm<double>(h, Ubra, Tp, out, false, true, stream);
}

void Engine::env_right_raw(int rb, int rk, int rb2, int rk2, int RB, const double* E, const double* Ubra,
                           const double* Uket, const SiteOp& w, int RA, double* out, const MixQ* q) {
  const long long sl = (long long)rk * 4 * rb2;
  ws2.ensure(sizeof(double) * sl * RB);
  ws3.ensure(sizeof(double) * sl * RA);
  double* T = ws2.as<double>();
  double* Tp = ws3.as<double>();
  GemmArgs g{};
  g.M = 4 * rk; g.N = rb2; g.K = rk2; g.batch = RB; g.kin = rk2;
  g.sAb = 0; g.sAm = rk2; g.sAkb = 0; g.sAkk = 1;
  g.sBb = (long long)rb2 * rk2; g.sBkb = 0; g.sBkk = 1; g.sBn = rk2;
  g.sCb = sl; g.sCm = rb2; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, Uket, E, T, true, false, stream);
  mix<double>(w.nout, w.ptr.as<int>(), w.src.as<int>(), w.op64.as<double>(), T, sl, Tp, sl, rk, rb2, stream, q);
  GemmArgs h{};
  h.M = rb; h.N = rk; h.K = 4 * rb2; h.batch = RA; h.kin = 4 * rb2;
  h.sAb = 0; h.sAm = 4LL * rb2; h.sAkb = 0; h.sAkk = 1;
  h.sBb = sl; h.sBkb = 0; h.sBkk = 1; h.sBn = 4LL * rb2;
  h.sCb = (long long)rb * rk; h.sCm = rk; h.alpha = 1.0; h.beta = 0.0;
  gemm<double>(h, Ubra, Tp, out, true, false, stream);
}

static inline int kin16(int K) { return ((K + 15) / 16) * 16; }

// The coefficient-block transform of environment slabs [bra r][ket c] (row length cp),
// restricted by charge: channel class d is non-zero only where q(bra r) - q(ket c) = d,
// and the block couples only channels of one class.  transpose=false:
// out[q][:] = sum_p V[q][p] in[p][:]; transpose=true: out[p][:] = sum_q V[q][p] in[q][:]
// (channel indices relative to the block).  Every other element of the nout output
// slabs is zero.
static void channel_transform_qn(Engine& E, const SiteMPO& s, const double* in, long long slab, double* out, int nout,
                                 const Labels& rq, const Labels& cq, int cp, bool transpose) {
  fill(out, sizeof(double) * slab * nout, E.stream);
  std::map<Q2, std::vector<int>> cols_of;
  for (int c = 0; c < (int)cq.size(); ++c) cols_of[cq[c]].push_back(c);
  for (const SiteMPO::VClass& c : s.vcls) {
    if (c.P.empty() || c.Q.empty()) continue;
    std::vector<int> pos;
    for (int r = 0; r < (int)rq.size(); ++r) {
      auto it = cols_of.find(qsub(rq[r], c.d));
      if (it == cols_of.end()) continue;
      for (int col : it->second) pos.push_back(r * cp + col);
    }
    if (pos.empty()) continue;
    if ((long long)rq.size() * cp > slab) throw std::runtime_error("channel transform: labels exceed the slab");
    const int np = (int)pos.size();
    const int nin = transpose ? (int)c.Q.size() : (int)c.P.size();
    const int nou = transpose ? (int)c.P.size() : (int)c.Q.size();
    const int* lin = transpose ? c.Qd.as<int>() : c.Pd.as<int>();
    const int* lout = transpose ? c.Pd.as<int>() : c.Qd.as<int>();
    DevMem pd = upload_ints(pos, E.stream);
    DevMem ci, co;
    ci.ensure(sizeof(double) * (size_t)nin * np);
    co.ensure(sizeof(double) * (size_t)nou * np);
    gather2d(in, slab, lin, nin, pd.as<int>(), np, ci.as<double>(), false, E.stream);
    GemmArgs g{};
    g.batch = 1; g.M = nou; g.N = np; g.K = nin; g.kin = kin16(nin); g.alpha = 1.0; g.beta = 0.0;
    g.sBb = 0; g.sBkb = 0; g.sBkk = np; g.sBn = 1; g.sCb = 0; g.sCm = np; g.sAb = 0; g.sAkb = 0;
    if (!transpose) {
      g.sAm = (long long)c.P.size(); g.sAkk = 1;  // V[q][p], row-major [|Q|][|P|]
      gemm<double>(g, c.V.as<double>(), ci.as<double>(), co.as<double>(), true, true, E.stream);
    } else {
      g.sAm = 1; g.sAkk = (long long)c.P.size();  // V^T
      gemm<double>(g, c.V.as<double>(), ci.as<double>(), co.as<double>(), false, true, E.stream);
    }
    scatter2d(co.as<double>(), np, 1, lout, nou, pd.as<int>(), np, out, slab, 1.0, nullptr, nullptr, 0, E.stream);
    HC(hipStreamSynchronize(E.stream));
  }
}


void Engine::env_unit(Env& e, int R) {
  e.R = R;
  e.rb = 1;
  e.rk = 1;
  e.d.resize_zero(sizeof(double) * e.elems(), stream);
  double one = 1.0;
  HC(hipMemcpyAsync(e.d.p, &one, sizeof(double), hipMemcpyHostToDevice, stream));
  HC(hipStreamSynchronize(stream));
}

// block-sparse left-update tables of a site (inputs: the channels of the left bond, then
// at a coefficient-block site the virtual channels standing for its block outputs);
// built once per MPO under the problem's mutex and shared by all engines
std::shared_ptr<BsSiteUse> Engine::left_site_use(int site) {
  SiteMPO& sm = mpo[site];
  std::lock_guard<std::mutex> g(prob->mu);
  if (!sm.bs_left) {
    std::vector<Q2> din(chan_q[site].begin(), chan_q[site].end());
    if (sm.has_block)
      for (int q = sm.q0; q < sm.q1; ++q) din.push_back(chan_q[site + 1][q]);
    std::vector<Q2> dout(chan_q[site + 1].begin(), chan_q[site + 1].end());
    auto u = std::make_shared<BsSiteUse>();
    bs_site_use(*this, *u, sm.has_block ? sm.byB_left : sm.byB, din, dout, +1);
    sm.bs_left = u;
  }
  return sm.bs_left;
}

void Engine::env_left(const Env& in, const Core& bra, const Core& ket, int site, Env& out) {
  const SiteMPO& s = mpo[site];
  if (in.R != s.Rl || in.rb != bra.rl || in.rk != ket.rl) throw std::runtime_error("env_left: shape mismatch");
  const int rb = padr(in.rb), rk = padr(in.rk), rb2 = bra.rrp(), rk2 = ket.rrp();
  Env o;
  o.R = s.Rr; o.rb = bra.rr; o.rk = ket.rr;
  o.d.ensure(sizeof(double) * o.elems());
  // mix output (B, a', s', b) can be non-zero only if q(s') = d_B - q(a') + q(b)
  MixQ q, *qp = nullptr;
  if (opts.qn_skip && (int)bra.ql.size() == bra.rl && (int)ket.qr.size() == ket.rr) {
    upload_q2(envq_o, padded_q(bra.ql, rb, 1), stream);
    upload_q2(envq_i, padded_q(ket.qr, rk2, -1), stream);
    q.qo = envq_o.as<int2>(); q.qi = envq_i.as<int2>(); q.qc = chan_q_dev[site + 1].as<int2>(); q.sgn = 1;
    qp = &q;
  }
  if (opts.qn_skip) {
    // block-sparse update (coefficient block handled through virtual input channels)
    std::shared_ptr<BsSiteUse> use = left_site_use(site);
    const double* Ein = in.d.as<double>();
    if (s.has_block) {
      const long long slab = (long long)rb * rk;
      const int nP = s.p1 - s.p0, nQ = s.q1 - s.q0;
      wsd.ensure(sizeof(double) * slab * (s.Rl + nQ));
      HC(hipMemcpyAsync(wsd.p, in.d.p, sizeof(double) * slab * s.Rl, hipMemcpyDeviceToDevice, stream));
      (void)nP;
      channel_transform_qn(*this, s, in.d.as<double>() + (long long)s.p0 * slab, slab,
                           wsd.as<double>() + (long long)s.Rl * slab, nQ, bra.ql, ket.ql, rk, false);
      Ein = wsd.as<double>();
    }
    bool done;
    {
      ScopeTimer tm(*this, t_env_bs, n_env_bs);
      done = bs_env(*this, *use, Ein, bra, ket, o.d.as<double>());
    }
    if (done) {
      out = std::move(o);
      return;
    }
  }
  ScopeTimer tmd(*this, t_env_dense, n_env_dense);
  if (s.has_block) {
    const long long slab = (long long)rb * rk;
    const int nP = s.p1 - s.p0, nQ = s.q1 - s.q0;
    wsd.ensure(sizeof(double) * slab * (s.Rl + nQ));
    HC(hipMemcpyAsync(wsd.p, in.d.p, sizeof(double) * slab * s.Rl, hipMemcpyDeviceToDevice, stream));
    (void)nP;
    channel_transform_qn(*this, s, in.d.as<double>() + (long long)s.p0 * slab, slab,
                         wsd.as<double>() + (long long)s.Rl * slab, nQ, bra.ql, ket.ql, rk, false);
    env_left_raw(rb, rk, rb2, rk2, s.Rl + nQ, wsd.as<double>(), bra.d.as<double>(), ket.d.as<double>(), s.byB_left,
                 s.Rr, o.d.as<double>(), qp);
  } else {
    env_left_raw(rb, rk, rb2, rk2, s.Rl, in.d.as<double>(), bra.d.as<double>(), ket.d.as<double>(), s.byB, s.Rr,
                 o.d.as<double>(), qp);
  }
  out = std::move(o);
}

void Engine::env_right(const Env& in, const Core& bra, const Core& ket, int site, Env& out) {
  const SiteMPO& s = mpo[site];
  if (in.R != s.Rr || in.rb != bra.rr || in.rk != ket.rr) throw std::runtime_error("env_right: shape mismatch");
  const int rb = bra.rlp(), rk = ket.rlp(), rb2 = padr(in.rb), rk2 = padr(in.rk);
  Env o;
  o.R = s.Rl; o.rb = bra.rl; o.rk = ket.rl;
  o.d.ensure(sizeof(double) * o.elems());
  // mix output (A, a, s', b') can be non-zero only if q(s') = q(b') - q(a) - d_A
  MixQ q, *qp = nullptr;
  if (opts.qn_skip && (int)ket.ql.size() == ket.rl && (int)bra.qr.size() == bra.rr) {
    upload_q2(envq_o, padded_q(ket.ql, rk, 1), stream);
    upload_q2(envq_i, padded_q(bra.qr, rb2, -1), stream);
    q.qo = envq_o.as<int2>(); q.qi = envq_i.as<int2>(); q.qc = chan_q_dev[site].as<int2>(); q.sgn = -1;
    qp = &q;
  }
  if (opts.qn_skip) {
    SiteMPO& sm = mpo[site];
    std::shared_ptr<BsSiteUse> use;
    {
      std::lock_guard<std::mutex> g(prob->mu);
      if (!sm.bs_right) {
        std::vector<Q2> din(chan_q[site + 1].begin(), chan_q[site + 1].end());
        if (sm.has_block)
          for (int p = sm.p0; p < sm.p1; ++p) din.push_back(chan_q[site][p]);
        std::vector<Q2> dout(chan_q[site].begin(), chan_q[site].end());
        auto u = std::make_shared<BsSiteUse>();
        bs_site_use(*this, *u, sm.has_block ? sm.byA_right : sm.byA, din, dout, -1);
        sm.bs_right = u;
      }
      use = sm.bs_right;
    }
    const double* Ein = in.d.as<double>();
    if (s.has_block) {
      const long long slab = (long long)rb2 * rk2;
      const int nP = s.p1 - s.p0, nQ = s.q1 - s.q0;
      wsd.ensure(sizeof(double) * slab * (s.Rr + nP));
      HC(hipMemcpyAsync(wsd.p, in.d.p, sizeof(double) * slab * s.Rr, hipMemcpyDeviceToDevice, stream));
      (void)nQ;
      channel_transform_qn(*this, s, in.d.as<double>() + (long long)s.q0 * slab, slab,
                           wsd.as<double>() + (long long)s.Rr * slab, nP, bra.qr, ket.qr, rk2, true);
      Ein = wsd.as<double>();
    }
    bool done;
    {
      ScopeTimer tm(*this, t_env_bs, n_env_bs);
      done = bs_env(*this, *use, Ein, bra, ket, o.d.as<double>());
    }
    if (done) {
      out = std::move(o);
      return;
    }
  }
  ScopeTimer tmd(*this, t_env_dense, n_env_dense);
  if (s.has_block) {
    const long long slab = (long long)rb2 * rk2;
    const int nP = s.p1 - s.p0, nQ = s.q1 - s.q0;
    wsd.ensure(sizeof(double) * slab * (s.Rr + nP));
    HC(hipMemcpyAsync(wsd.p, in.d.p, sizeof(double) * slab * s.Rr, hipMemcpyDeviceToDevice, stream));
    (void)nQ;
    channel_transform_qn(*this, s, in.d.as<double>() + (long long)s.q0 * slab, slab,
                         wsd.as<double>() + (long long)s.Rr * slab, nP, bra.qr, ket.qr, rk2, true);
    env_right_raw(rb, rk, rb2, rk2, s.Rr + nP, wsd.as<double>(), bra.d.as<double>(), ket.d.as<double>(), s.byA_right,
                  s.Rl, o.d.as<double>(), qp);
  } else {
    env_right_raw(rb, rk, rb2, rk2, s.Rr, in.d.as<double>(), bra.d.as<double>(), ket.d.as<double>(), s.byA, s.Rl,
                  o.d.as<double>(), qp);
  }
  out = std::move(o);
}

double Engine::env_close(const Env& Lb, const Env& Rb_) {
  if (Lb.R != Rb_.R || Lb.rb != Rb_.rb || Lb.rk != Rb_.rk) throw std::runtime_error("env_close: shape mismatch");
  const size_t n = Lb.elems();
  wsp.ensure(sizeof(double) * (256 + 8));
  DevMem part;
  part.ensure(sizeof(double) * kDotBlocks);
  multi_dot(Lb.d.as<double>(), n, 1, Rb_.d.as<double>(), n, wsp.as<double>(), part.as<double>(), kDotBlocks, stream);
  double v = 0.0;
  d2h(&v, wsp.p, sizeof(double), stream);
  return v;
}

// ---------------------------------------------------------------------------
// sector-wise linear algebra (rocSOLVER per charge block)
// ---------------------------------------------------------------------------
struct Sector {
  Q2 g;
  std::vector<int> rows, cols;
};

static std::vector<Sector> make_sectors(const std::vector<int>& rows, const Labels& rq, const std::vector<int>& cols,
                                        const Labels& cq) {
  std::map<Q2, Sector> m;
  for (size_t i = 0; i < rows.size(); ++i) {
    auto& s = m[rq[i]];
    s.g = rq[i];
    s.rows.push_back(rows[i]);
  }
  std::map<Q2, std::vector<int>> cm;
  for (size_t j = 0; j < cols.size(); ++j) cm[cq[j]].push_back(cols[j]);
  std::vector<Sector> out;
  for (auto& kv : m) {
    auto it = cm.find(kv.first);
    if (it == cm.end()) continue;
    kv.second.cols = it->second;
    out.push_back(kv.second);
  }
  return out;
}

static int truncation_keep(const std::vector<double>& sv, int chi, double cutoff, double tau) {
  if (sv.empty() || sv[0] <= 0.0) return 0;
  const double smax = sv[0];
  int n = 0;
  for (double s : sv)
    if (s >= cutoff * smax) ++n;
  if (n <= chi) return n;
  const double ref = sv[chi - 1];
  int gmin = -1, gmax = -1;
  for (int i = 0; i < n; ++i)
    if (std::fabs(sv[i] - ref) <= tau * smax) {
      if (gmin < 0) gmin = i;
      gmax = i;
    }
  if (gmin >= 0 && gmin < chi && gmax >= chi) return gmin;
  return chi;
}

struct SvdOut {
  int k = 0;
  Labels q;
  double discarded = 0.0;
  std::vector<double> s;
};

// Truncated SVD of the matrix M (device, element (r,c) at M[r*ldm + c]) restricted
// to the listed rows/cols, block-diagonal by charge.  Writes the left factor
// into left[r*ldl + j] and the right factor into right[j*ldr + c] (both
// pre-zeroed by the caller after the first pass, see two-phase use below).
// mode 0: right factor carries the singular values; mode 1: left factor.
// sweep limit of the Jacobi SVD kernel (a sweep visits every column pair once; the
// factorisations here converge in about ten)
constexpr int kJacobiSweeps = 40;
// blocks of at least this many columns go to the blocked Jacobi kernels (svd_blocked = 1)
constexpr int kJacobiBlockedMinN = 48;

class SectorSVD {
 public:
  SectorSVD(Engine& e) : E(e) {}
  SvdOut run(const double* M, long long ldm, const std::vector<int>& rows, const Labels& rq,
             const std::vector<int>& cols, const Labels& cq, int chi, bool truncate) {
    secs = make_sectors(rows, rq, cols, cq);
    const int ns = (int)secs.size();
    blocks.clear();
    blocks.resize(ns);
    bins.clear();
    // all sector indices in one upload; blocks binned by size into zero-padded storage of
    // the bin's largest block (the Jacobi kernel factors each block at its own size; a bin
    // too wide for it goes to one batched rocSOLVER SVD, whose top min(m, n) triplets of a
    // zero-padded block are those of the block).  Wide blocks (m < n) are factorised
    // transposed so that every matrix is tall.
    std::vector<int> allr, allc;
    std::map<long long, std::vector<int>> bykey;
    for (int t = 0; t < ns; ++t) {
      Blk& b = blocks[t];
      b.m = (int)secs[t].rows.size();
      b.n = (int)secs[t].cols.size();
      b.k = std::min(b.m, b.n);
      b.roff = (int)allr.size();
      b.coff = (int)allc.size();
      allr.insert(allr.end(), secs[t].rows.begin(), secs[t].rows.end());
      allc.insert(allc.end(), secs[t].cols.begin(), secs[t].cols.end());
      b.tr = b.m < b.n;
      int key = 16;
      while (key < std::max(b.m, b.n)) key *= 2;
      bykey[key].push_back(t);
    }
    rdev = upload_ints(allr, E.stream);
    cdev = upload_ints(allc, E.stream);
    struct Trip {
      double s;
      Q2 g;
      int sec, i;
    };
    std::vector<Trip> trip;
    // phase 1 (context stream): padded bins gathered
    std::vector<const std::vector<int>*> members;
    for (auto& kv : bykey) {
      bins.emplace_back();
      Bin& B = bins.back();
      const std::vector<int>& mem = kv.second;
      members.push_back(&mem);
      B.cnt = (int)mem.size();
      for (int t : mem) {
        B.M = std::max(B.M, std::max(blocks[t].m, blocks[t].n));
        B.N = std::max(B.N, std::min(blocks[t].m, blocks[t].n));
      }
      B.K = B.N;
      const long long MN = (long long)B.M * B.N;
      B.A.ensure(sizeof(double) * MN * B.cnt);
      // the zero padding matters only to the batched rocSOLVER path (bins wider than the
      // Jacobi kernel takes); the kernel reads each block at its own size
      if (B.N > kJacobiMaxN) fill(B.A.p, sizeof(double) * MN * B.cnt, E.stream);
      std::vector<GatherBlk> gb(B.cnt);
      for (int i = 0; i < B.cnt; ++i) {
        const Blk& b = blocks[mem[i]];
        gb[i] = GatherBlk{MN * i, B.M, b.roff, b.coff, b.m, b.n, b.tr ? 1 : 0};
      }
      upload(B.gdev, gb.data(), gb.size() * sizeof(GatherBlk), E.stream);
      gather_blocks(M, ldm, rdev.as<int>(), cdev.as<int>(), B.gdev.as<GatherBlk>(), B.cnt, B.A.as<double>(), E.stream);
      B.U.ensure(sizeof(double) * (size_t)B.M * B.K * B.cnt);
      B.Vt.ensure(sizeof(double) * (size_t)B.K * B.N * B.cnt);
      B.S.ensure(sizeof(double) * (size_t)B.K * B.cnt);
      B.Ew.ensure(sizeof(double) * (size_t)B.K * B.cnt);
      B.info.ensure(sizeof(int) * B.cnt);
    }
    HC(hipStreamSynchronize(E.stream));
    // phase 2: every block in one launch of the Jacobi SVD kernel at its own size (tall:
    // M = max(m, n), N = min(m, n)), in the storage of its bin, held in LDS where it fits;
    // bins wider than the kernel takes go to rocSOLVER whole
    auto factor = [&](Bin& B, rocblas_handle h) {
      const long long MN = (long long)B.M * B.N;
      RC(rocsolver_dgesvd_strided_batched(h, rocblas_svect_singular, rocblas_svect_singular, B.M, B.N,
                                          B.A.as<double>(), B.M, MN, B.S.as<double>(), B.K, B.U.as<double>(), B.M,
                                          (rocblas_stride)B.M * B.K, B.Vt.as<double>(), B.K, (rocblas_stride)B.K * B.N,
                                          B.Ew.as<double>(), B.K, rocblas_outofplace, B.info.as<int>(), B.cnt));
    };
    const double tb0 = E.verbose ? E.now() : 0.0;
    {
      // the one-workgroup kernel (global memory, or LDS where the block fits) or, for wide
      // blocks, the blocked kernels
      auto blocked = [&](int m, int n) {
        const int mode = E.opts.svd_blocked;
        return mode != 0 && n >= (mode == 1 ? kJacobiBlockedMinN : 2) && jacobi_blocked_fits(m, n);
      };
      std::vector<SvdJob> jobs[2], bjobs;
      long long vtot = 0;
      for (size_t bi = 0; bi < bins.size(); ++bi) {
        if (bins[bi].N > kJacobiMaxN) continue;
        for (int t : *members[bi]) {
          const long long m = std::max(blocks[t].m, blocks[t].n), n = std::min(blocks[t].m, blocks[t].n);
          if (blocked((int)m, (int)n) || !E.opts.svd_lds || (m + n) * n > kJacobiLds) vtot += n * n;
        }
      }
      DevMem Vs, jdev[2], bdev, bscr;
      Vs.ensure(sizeof(double) * (size_t)std::max<long long>(vtot, 1));
      long long voff = 0;
      for (size_t bi = 0; bi < bins.size(); ++bi) {
        Bin& B = bins[bi];
        if (B.N > kJacobiMaxN) continue;
        const std::vector<int>& mem = *members[bi];
        for (int i = 0; i < B.cnt; ++i) {
          const Blk& b = blocks[mem[i]];
          const int m = std::max(b.m, b.n), n = std::min(b.m, b.n);
          const bool bj = blocked(m, n);
          const int in_lds = !bj && E.opts.svd_lds && (long long)(m + n) * n <= kJacobiLds ? 1 : 0;
          const SvdJob job{B.A.as<double>() + (size_t)B.M * B.N * i, in_lds ? nullptr : Vs.as<double>() + voff,
                           B.U.as<double>() + (size_t)B.M * B.K * i, B.S.as<double>() + (size_t)B.K * i,
                           B.Vt.as<double>() + (size_t)B.K * B.N * i, B.info.as<int>() + i, m, n, B.M, B.M,
                           B.K, 0};
          if (bj) bjobs.push_back(job);
          else jobs[in_lds].push_back(job);
          if (!in_lds) voff += (long long)n * n;
        }
      }
      for (int v = 0; v < 2; ++v)
        if (!jobs[v].empty()) {
          upload(jdev[v], jobs[v].data(), jobs[v].size() * sizeof(SvdJob), E.stream);
          jacobi_svd(jdev[v].as<SvdJob>(), (int)jobs[v].size(), kJacobiSweeps, v == 1, E.stream);
        }
      if (!bjobs.empty()) {
        const size_t nj = bjobs.size();
        upload(bdev, bjobs.data(), nj * sizeof(SvdJob), E.stream);
        // per matrix: |A|_F^2 (double), rotation count and active index (int)
        bscr.ensure(nj * (sizeof(double) + 2 * sizeof(int)));
        double* fro2 = bscr.as<double>();
        int* rot = reinterpret_cast<int*>(fro2 + nj);
        // svd_blocked 3 and 4 pin the pair kernels' rows per lane (loops over LDS, or 9)
        const int rows = E.opts.svd_blocked == 3 ? 0 : E.opts.svd_blocked == 4 ? 9 : -1;
        jacobi_svd_blocked(bdev.as<SvdJob>(), bjobs.data(), (int)nj, rows, kJacobiSweeps, fro2, rot, rot + nj,
                           E.stream);
      }
      for (Bin& B : bins)
        if (B.N > kJacobiMaxN) factor(B, E.blas);
      HC(hipStreamSynchronize(E.stream));
    }
    if (E.verbose) {
      const double dt = E.now() - tb0;
      for (Bin& B : bins) {
        auto& st = E.svd_bins[{B.M, B.N}];
        st[0] += 1.0;
        st[1] += B.cnt;
      }
      E.svd_seconds += dt;
    }
    // phase 3 (context stream): convergence check, singular triplets
    for (size_t bi = 0; bi < bins.size(); ++bi) {
      Bin& B = bins[bi];
      const std::vector<int>& mem = *members[bi];
      std::vector<int> inf(B.cnt);
      d2h(inf.data(), B.info.p, sizeof(int) * B.cnt, E.stream);
      for (int i = 0; i < B.cnt; ++i) {
        if (inf[i] == 0) continue;
        // a block whose factorisation did not converge (or a shape the Jacobi kernel does
        // not take) is factored again by rocSOLVER at its own size, into its slots of the bin
        const Blk& bb = blocks[mem[i]];
        {
          const int mm = std::max(bb.m, bb.n), nn = std::min(bb.m, bb.n);
          DevMem a1, e1, i1;
          a1.ensure(sizeof(double) * (size_t)mm * nn);
          e1.ensure(sizeof(double) * std::max(nn, 1));
          i1.ensure(sizeof(int));
          GatherBlk one{0, mm, bb.roff, bb.coff, bb.m, bb.n, bb.tr ? 1 : 0};
          DevMem odev;
          upload(odev, &one, sizeof(one), E.stream);
          gather_blocks(M, ldm, rdev.as<int>(), cdev.as<int>(), odev.as<GatherBlk>(), 1, a1.as<double>(), E.stream);
          RC(rocsolver_dgesvd(E.blas, rocblas_svect_singular, rocblas_svect_singular, mm, nn, a1.as<double>(), mm,
                              B.S.as<double>() + (size_t)B.K * i, B.U.as<double>() + (size_t)B.M * B.K * i, B.M,
                              B.Vt.as<double>() + (size_t)B.K * B.N * i, B.K, e1.as<double>(), rocblas_outofplace,
                              i1.as<int>()));
          d2h(&inf[i], i1.p, sizeof(int), E.stream);
        }
        if (inf[i] != 0) {
          const Blk& b = blocks[mem[i]];
          // describe the input block (the gathered copy was overwritten by the factorisation)
          std::vector<double> hb((size_t)b.m * b.n);
          {
            DevMem tmp;
            tmp.ensure(sizeof(double) * hb.size());
            GatherBlk one{0, b.m, b.roff, b.coff, b.m, b.n, 0};
            DevMem odev;
            upload(odev, &one, sizeof(one), E.stream);
            gather_blocks(M, ldm, rdev.as<int>(), cdev.as<int>(), odev.as<GatherBlk>(), 1, tmp.as<double>(),
                          E.stream);
            d2h(hb.data(), tmp.p, sizeof(double) * hb.size(), E.stream);
          }
          double mx = 0.0;
          int nonfinite = 0;
          for (double v : hb) {
            if (!std::isfinite(v)) ++nonfinite;
            else mx = std::max(mx, std::fabs(v));
          }
          std::string vals;
          for (size_t q = 0; q < std::min<size_t>(hb.size(), 8); ++q) vals += " " + std::to_string(hb[q]);
          throw std::runtime_error("gesvd did not converge (info " + std::to_string(inf[i]) + ", block " +
                                   std::to_string(b.m) + "x" + std::to_string(b.n) + " padded to " +
                                   std::to_string(B.M) + "x" + std::to_string(B.N) + ", batch " +
                                   std::to_string(B.cnt) + ", max|a| " + std::to_string(mx) + ", non-finite " +
                                   std::to_string(nonfinite) + ", first:" + vals + ")");
        }
      }
      std::vector<double> hs((size_t)B.K * B.cnt);
      d2h(hs.data(), B.S.p, sizeof(double) * hs.size(), E.stream);
      for (int i = 0; i < B.cnt; ++i) {
        const int t = mem[i];
        Blk& b = blocks[t];
        const double* Ub = B.U.as<double>() + (size_t)B.M * B.K * i;   // B.M x B.K, column-major
        const double* Vb = B.Vt.as<double>() + (size_t)B.K * B.N * i;  // B.K x B.N, column-major
        b.S = B.S.as<double>() + (size_t)B.K * i;
        if (!b.tr) {
          // A = U S V^T: U[i][j] = Ub[i + j*M], V^T[j][c] = Vb[j + c*K]
          b.U = Ub; b.us_i = 1; b.us_j = B.M;
          b.Vt = Vb; b.vs_j = 1; b.vs_c = B.K;
        } else {
          // A^T = U' S V'^T, so A = V' S U'^T: U[i][j] = V'^T[j][i], V^T[j][c] = U'[c][j]
          b.U = Vb; b.us_i = B.K; b.us_j = 1;
          b.Vt = Ub; b.vs_j = B.M; b.vs_c = 1;
        }
        b.hs.assign(hs.begin() + (size_t)B.K * i, hs.begin() + (size_t)B.K * i + b.k);
        for (int q = 0; q < b.k; ++q) trip.push_back({b.hs[q], secs[t].g, t, q});
      }
    }
    std::sort(trip.begin(), trip.end(), [](const Trip& a, const Trip& b) {
      if (a.s != b.s) return a.s > b.s;
      if (a.g != b.g) return a.g < b.g;
      return a.i < b.i;
    });
    std::vector<double> all(trip.size());
    for (size_t i = 0; i < trip.size(); ++i) all[i] = trip[i].s;
    // truncate: R7 rule; otherwise every singular triplet is kept (orthogonal factorisations)
    const int keep = truncate ? truncation_keep(all, chi, E.opts.svd_cutoff, E.opts.tie_rel) : (int)all.size();
    SvdOut out;
    for (size_t i = keep; i < all.size(); ++i) out.discarded += all[i] * all[i];
    std::vector<int> cnt(secs.size(), 0);
    for (int i = 0; i < keep; ++i) cnt[trip[i].sec]++;
    // new bond order: sectors in charge order (make_sectors returns sorted), then decreasing s
    int off = 0;
    for (size_t t = 0; t < secs.size(); ++t) {
      blocks[t].t = cnt[t];
      blocks[t].off = off;
      for (int i = 0; i < cnt[t]; ++i) {
        out.q.push_back(secs[t].g);
        out.s.push_back(blocks[t].hs[i]);
      }
      off += cnt[t];
    }
    out.k = off;
    return out;
  }
  // scatter the kept factors (destination arrays must be zero initialised)
  void scatter(double* left, long long ldl, double* right, long long ldr, int mode) {
    std::vector<ScatterBlk> sb;
    for (const Blk& b : blocks)
      if (b.t > 0)
        sb.push_back(ScatterBlk{b.U, b.Vt, b.S, b.us_i, b.us_j, b.vs_j, b.vs_c, b.roff, b.coff, b.m, b.n, b.t, b.off});
    if (!sb.empty()) {
      DevMem sdev;
      upload(sdev, sb.data(), sb.size() * sizeof(ScatterBlk), E.stream);
      scatter_factors(sdev.as<ScatterBlk>(), (int)sb.size(), rdev.as<int>(), cdev.as<int>(), left, ldl, right, ldr,
                      mode, E.stream);
    }
    HC(hipStreamSynchronize(E.stream));
  }

 private:
  Engine& E;
  struct Blk {
    int m = 0, n = 0, k = 0, t = 0, off = 0, roff = 0, coff = 0;
    bool tr = false;                  // factorised transposed (wide block)
    long long us_i = 0, us_j = 0, vs_j = 0, vs_c = 0;  // element strides of U and V^T
    const double* U = nullptr;
    const double* Vt = nullptr;
    const double* S = nullptr;
    std::vector<double> hs;
  };
  struct Bin {
    int M = 0, N = 0, K = 0, cnt = 0;
    DevMem A, U, Vt, S, Ew, info, gdev;
  };
  std::vector<Sector> secs;
  std::vector<Blk> blocks;
  std::vector<Bin> bins;
  DevMem rdev, cdev;
};

// QR of core A viewed as [(a s)][b]; A <- Q (left-orthogonal), next <- R next.
static void qr_left_solver(Engine& E, Core& A, Core& next) {
  const int rlp = A.rlp(), rrp = A.rrp();
  std::vector<int> rows, cols;
  Labels rq, cq;
  for (int a = 0; a < A.rl; ++a)
    for (int s = 0; s < 4; ++s) {
      rows.push_back(a * 4 + s);
      rq.push_back(qadd(A.ql[a], SITE_Q[s]));
    }
  for (int b = 0; b < A.rr; ++b) {
    cols.push_back(b);
    cq.push_back(A.qr[b]);
  }
  // every column must belong to a sector with at least as many rows
  auto secs = make_sectors(rows, rq, cols, cq);
  size_t ncov = 0;
  for (auto& s : secs) {
    if (s.rows.size() < s.cols.size()) throw std::runtime_error("rank-deficient QN block in QR");
    ncov += s.cols.size();
  }
  if (ncov != cols.size()) throw std::runtime_error("TT core has a bond state with no compatible rows");
  DevMem Qd, Rm;
  Qd.resize_zero(sizeof(double) * (size_t)rlp * 4 * rrp, E.stream);
  Rm.resize_zero(sizeof(double) * (size_t)rrp * rrp, E.stream);
  DevMem info, tau;
  info.ensure(sizeof(int));
  for (auto& sc : secs) {
    const int m = (int)sc.rows.size(), n = (int)sc.cols.size();
    DevMem blk, rdev = upload_ints(sc.rows, E.stream), cdev = upload_ints(sc.cols, E.stream);
    blk.ensure(sizeof(double) * m * n);
    tau.ensure(sizeof(double) * n);
    gather2d(A.d.as<double>(), rrp, rdev.as<int>(), m, cdev.as<int>(), n, blk.as<double>(), true, E.stream);
    RC(rocsolver_dgeqrf(E.blas, m, n, blk.as<double>(), m, tau.as<double>()));
    // R (upper n x n) -> Rm[cols][cols]
    scatter2d(blk.as<double>(), 1, m, cdev.as<int>(), n, cdev.as<int>(), n, Rm.as<double>(), rrp, 1.0, nullptr,
              nullptr, 1, E.stream);
    RC(rocsolver_dorgqr(E.blas, m, n, n, blk.as<double>(), m, tau.as<double>()));
    scatter2d(blk.as<double>(), 1, m, rdev.as<int>(), m, cdev.as<int>(), n, Qd.as<double>(), rrp, 1.0, nullptr,
              nullptr, 0, E.stream);
    HC(hipStreamSynchronize(E.stream));
  }
  A.d = std::move(Qd);
  // next <- Rm * next : [rrp][rrp] x [rrp][4*nrp]
  const int nrp = next.rrp();
  DevMem nd;
  nd.ensure(sizeof(double) * (size_t)rrp * 4 * nrp);
  GemmArgs g{};
  g.M = rrp; g.N = 4 * nrp; g.K = rrp; g.batch = 1; g.kin = rrp;
  g.sAm = rrp; g.sAkk = 1; g.sBkk = 4LL * nrp; g.sBn = 1; g.sCm = 4LL * nrp; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, Rm.as<double>(), next.d.as<double>(), nd.as<double>(), true, true, E.stream);
  HC(hipStreamSynchronize(E.stream));
  next.d = std::move(nd);
}

// LQ of core W viewed as [a][(s b)]: W <- Q (right-orthogonal, possibly smaller
// left bond), prev <- prev Lmat.  Returns the new left labels.
static void lq_right_solver(Engine& E, Core& W, Core& prev) {
  const int rlp = W.rlp(), rrp = W.rrp();
  std::vector<int> rows, cols;
  Labels rq, cq;
  for (int a = 0; a < W.rl; ++a) {
    rows.push_back(a);
    rq.push_back(W.ql[a]);
  }
  for (int s = 0; s < 4; ++s)
    for (int b = 0; b < W.rr; ++b) {
      cols.push_back(s * rrp + b);
      cq.push_back(qsub(W.qr[b], SITE_Q[s]));
    }
  auto secs = make_sectors(rows, rq, cols, cq);
  // new left bond: k_g = min(m_g, n_g) per sector, in charge order
  int knew = 0;
  Labels qn;
  std::vector<int> offs;
  for (auto& sc : secs) {
    int k = (int)std::min(sc.rows.size(), sc.cols.size());
    offs.push_back(knew);
    for (int i = 0; i < k; ++i) qn.push_back(sc.g);
    knew += k;
  }
  const int kp = padr(knew);
  DevMem Qd, Lm;
  Qd.resize_zero(sizeof(double) * (size_t)kp * 4 * rrp, E.stream);
  Lm.resize_zero(sizeof(double) * (size_t)rlp * kp, E.stream);
  DevMem tau;
  for (size_t t = 0; t < secs.size(); ++t) {
    auto& sc = secs[t];
    const int m = (int)sc.rows.size(), n = (int)sc.cols.size(), k = std::min(m, n);
    DevMem blk, rdev = upload_ints(sc.rows, E.stream), cdev = upload_ints(sc.cols, E.stream);
    std::vector<int> nidx(k);
    std::iota(nidx.begin(), nidx.end(), offs[t]);
    DevMem ndev = upload_ints(nidx, E.stream);
    blk.ensure(sizeof(double) * m * n);
    tau.ensure(sizeof(double) * k);
    gather2d(W.d.as<double>(), 4LL * rrp, rdev.as<int>(), m, cdev.as<int>(), n, blk.as<double>(), true, E.stream);
    RC(rocsolver_dgelqf(E.blas, m, n, blk.as<double>(), m, tau.as<double>()));
    // L: lower trapezoid m x k -> Lm[rows][new]
    scatter2d(blk.as<double>(), 1, m, rdev.as<int>(), m, ndev.as<int>(), k, Lm.as<double>(), kp, 1.0, nullptr,
              nullptr, 2, E.stream);
    RC(rocsolver_dorglq(E.blas, k, n, k, blk.as<double>(), m, tau.as<double>()));
    // Q: k x n (leading k rows of the m x n array, ld m) -> Qd[new][cols]
    scatter2d(blk.as<double>(), 1, m, ndev.as<int>(), k, cdev.as<int>(), n, Qd.as<double>(), 4LL * rrp, 1.0,
              nullptr, nullptr, 0, E.stream);
    HC(hipStreamSynchronize(E.stream));
  }
  W.d = std::move(Qd);
  W.rl = knew;
  W.ql = qn;
  // prev [prlp][4][rlp] x Lm [rlp][kp] -> [prlp][4][kp]
  const int prlp = prev.rlp();
  DevMem nd;
  nd.ensure(sizeof(double) * (size_t)prlp * 4 * kp);
  GemmArgs g{};
  g.M = prlp * 4; g.N = kp; g.K = rlp; g.batch = 1; g.kin = rlp;
  g.sAm = rlp; g.sAkk = 1; g.sBkk = kp; g.sBn = 1; g.sCm = kp; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, prev.d.as<double>(), Lm.as<double>(), nd.as<double>(), true, true, E.stream);
  HC(hipStreamSynchronize(E.stream));
  prev.d = std::move(nd);
  prev.rr = knew;
  prev.qr = qn;
}

// All sector blocks of one orthogonal factorisation in one launch of the
// Householder kernel (one workgroup per block).
struct HhJob {
  std::vector<int> rows, cols, nmap;
  std::vector<HhBlk> blks;
  long long ws = 0;
  int maxn = 0;
  void add(const std::vector<int>& r, const std::vector<int>& c, const std::vector<int>& nm) {
    const int m = (int)r.size(), n = (int)c.size(), k = std::min(m, n);
    if ((int)nm.size() != k) throw std::logic_error("Householder job: factor index map size");
    blks.push_back(HhBlk{ws, m, n, (int)rows.size(), (int)cols.size(), (int)nmap.size(), 0});
    rows.insert(rows.end(), r.begin(), r.end());
    cols.insert(cols.end(), c.begin(), c.end());
    nmap.insert(nmap.end(), nm.begin(), nm.end());
    ws += (long long)m * n + (long long)k * n + k;
    maxn = std::max(maxn, n);
  }
  void run(Engine& E, const double* W, long long sWr, long long sWc, double* L, long long sLr, long long sLc, double* Q,
           long long sQr, long long sQc) {
    if (blks.empty()) return;
    DevMem dr = upload_ints(rows, E.stream), dc = upload_ints(cols, E.stream), dn = upload_ints(nmap, E.stream);
    DevMem db, dws;
    upload(db, blks.data(), blks.size() * sizeof(HhBlk), E.stream);
    dws.ensure(sizeof(double) * std::max<long long>(ws, 1));
    householder_lq(W, sWr, sWc, dr.as<int>(), dc.as<int>(), dn.as<int>(), db.as<HhBlk>(), (int)blks.size(),
                   dws.as<double>(), L, sLr, sLc, Q, sQr, sQc, E.stream);
    HC(hipStreamSynchronize(E.stream));
  }
};

// QR of core A viewed as [(a s)][b] per charge sector: A <- Q (left-orthogonal, same
// bond basis), next <- R next.  Computed as the LQ of the transposed blocks.
static void qr_left(Engine& E, Core& A, Core& next) {
  const int rlp = A.rlp(), rrp = A.rrp();
  std::vector<int> rows, cols;
  Labels rq, cq;
  for (int a = 0; a < A.rl; ++a)
    for (int s = 0; s < 4; ++s) {
      rows.push_back(a * 4 + s);
      rq.push_back(qadd(A.ql[a], SITE_Q[s]));
    }
  for (int b = 0; b < A.rr; ++b) {
    cols.push_back(b);
    cq.push_back(A.qr[b]);
  }
  // every column must belong to a sector with at least as many rows
  auto secs = make_sectors(rows, rq, cols, cq);
  size_t ncov = 0;
  HhJob J;
  for (auto& sc : secs) {
    if (sc.rows.size() < sc.cols.size()) throw std::runtime_error("rank-deficient QN block in QR");
    ncov += sc.cols.size();
    J.add(sc.cols, sc.rows, sc.cols);
  }
  if (ncov != cols.size()) throw std::runtime_error("TT core has a bond state with no compatible rows");
  if (J.maxn > HH_MAXN) {
    qr_left_solver(E, A, next);
    return;
  }
  DevMem Qd, Rm;
  Qd.resize_zero(sizeof(double) * (size_t)rlp * 4 * rrp, E.stream);
  Rm.resize_zero(sizeof(double) * (size_t)rrp * rrp, E.stream);
  // transposed block [b][(a s)] = A[(a s)][b]; R[b'][b] = L^T; Q[(a s)][b'] = Q'^T
  J.run(E, A.d.as<double>(), 1, rrp, Rm.as<double>(), 1, rrp, Qd.as<double>(), 1, rrp);
  A.d = std::move(Qd);
  // next <- Rm * next : [rrp][rrp] x [rrp][4*nrp]
  const int nrp = next.rrp();
  DevMem nd;
  nd.ensure(sizeof(double) * (size_t)rrp * 4 * nrp);
  GemmArgs g{};
  g.M = rrp; g.N = 4 * nrp; g.K = rrp; g.batch = 1; g.kin = rrp;
  g.sAm = rrp; g.sAkk = 1; g.sBkk = 4LL * nrp; g.sBn = 1; g.sCm = 4LL * nrp; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, Rm.as<double>(), next.d.as<double>(), nd.as<double>(), true, true, E.stream);
  HC(hipStreamSynchronize(E.stream));
  next.d = std::move(nd);
}

// W = L Q with W viewed as [a][(s b)] per charge sector: W <- Q (right-orthogonal, left
// bond k_g = min(m_g, n_g) per sector, in charge order), prev <- prev L.
static void lq_right(Engine& E, Core& W, Core& prev) {
  const int rlp = W.rlp(), rrp = W.rrp();
  std::vector<int> rows, cols;
  Labels rq, cq;
  for (int a = 0; a < W.rl; ++a) {
    rows.push_back(a);
    rq.push_back(W.ql[a]);
  }
  for (int s = 0; s < 4; ++s)
    for (int b = 0; b < W.rr; ++b) {
      cols.push_back(s * rrp + b);
      cq.push_back(qsub(W.qr[b], SITE_Q[s]));
    }
  auto secs = make_sectors(rows, rq, cols, cq);
  int knew = 0;
  Labels qn;
  HhJob J;
  for (auto& sc : secs) {
    const int k = (int)std::min(sc.rows.size(), sc.cols.size());
    std::vector<int> nm(k);
    std::iota(nm.begin(), nm.end(), knew);
    for (int i = 0; i < k; ++i) qn.push_back(sc.g);
    knew += k;
    J.add(sc.rows, sc.cols, nm);
  }
  if (J.maxn > HH_MAXN) {
    lq_right_solver(E, W, prev);
    return;
  }
  const int kp = padr(std::max(knew, 1));
  DevMem Qd, Lm;
  Qd.resize_zero(sizeof(double) * (size_t)kp * 4 * rrp, E.stream);
  Lm.resize_zero(sizeof(double) * (size_t)rlp * kp, E.stream);
  J.run(E, W.d.as<double>(), 4LL * rrp, 1, Lm.as<double>(), kp, 1, Qd.as<double>(), 4LL * rrp, 1);
  W.d = std::move(Qd);
  W.rl = knew;
  W.ql = qn;
  // prev [prlp][4][rlp] x Lm [rlp][kp] -> [prlp][4][kp]
  const int prlp = prev.rlp();
  DevMem nd;
  nd.ensure(sizeof(double) * (size_t)prlp * 4 * kp);
  GemmArgs g{};
  g.M = prlp * 4; g.N = kp; g.K = rlp; g.batch = 1; g.kin = rlp;
  g.sAm = rlp; g.sAkk = 1; g.sBkk = kp; g.sBn = 1; g.sCm = kp; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, prev.d.as<double>(), Lm.as<double>(), nd.as<double>(), true, true, E.stream);
  HC(hipStreamSynchronize(E.stream));
  prev.d = std::move(nd);
  prev.rr = knew;
  prev.qr = qn;
}

// two-site tensor x[a][s1][s2][b] = sum_k C[a][s1][k] D[k][s2][b]
static void two_site(Engine& E, const Core& C, const Core& D, DevMem& x) {
  const int rlp = C.rlp(), kp = C.rrp(), rrp = D.rrp();
  if (C.rr != D.rl) throw std::runtime_error("two_site: bond mismatch");
  x.ensure(sizeof(double) * (size_t)rlp * 16 * rrp);
  GemmArgs g{};
  g.M = 4 * rlp; g.N = 4 * rrp; g.K = kp; g.batch = 1; g.kin = kp;
  g.sAm = kp; g.sAkk = 1; g.sBkk = 4LL * rrp; g.sBn = 1; g.sCm = 4LL * rrp; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, C.d.as<double>(), D.d.as<double>(), x.as<double>(), true, true, E.stream);
}

// split x (padded [rlp][4][4][rrp]) by the truncated block SVD into (N, C) with
// labels; left_normal: N left-orthogonal, C = S V^T; else N = U S, C = V^T.
static double split_two_site(Engine& E, const double* x, int rl, const Labels& ql, int rr, const Labels& qr, int chi,
                             bool left_normal, Core& N, Core& C) {
  const int rlp = padr(rl), rrp = padr(rr);
  std::vector<int> rows, cols;
  Labels rq, cq;
  for (int a = 0; a < rl; ++a)
    for (int s = 0; s < 4; ++s) {
      rows.push_back(a * 4 + s);
      rq.push_back(qadd(ql[a], SITE_Q[s]));
    }
  for (int s = 0; s < 4; ++s)
    for (int b = 0; b < rr; ++b) {
      cols.push_back(s * rrp + b);
      cq.push_back(qsub(qr[b], SITE_Q[s]));
    }
  SectorSVD svd(E);
  SvdOut o = svd.run(x, 4LL * rrp, rows, rq, cols, cq, chi, true);
  const int k = o.k, kp = padr(std::max(k, 1));
  N.rl = rl; N.ql = ql; N.rr = k; N.qr = o.q;
  C.rl = k; C.ql = o.q; C.rr = rr; C.qr = qr;
  N.d.resize_zero(sizeof(double) * (size_t)rlp * 4 * kp, E.stream);
  C.d.resize_zero(sizeof(double) * (size_t)kp * 4 * rrp, E.stream);
  svd.scatter(N.d.as<double>(), kp, C.d.as<double>(), 4LL * rrp, left_normal ? 0 : 1);
  return o.discarded;
}

static double norm_dev(Engine& E, const double* x, size_t n) {
  DevMem out, part;
  out.ensure(sizeof(double));
  part.ensure(sizeof(double) * kDotBlocks);
  multi_dot(x, n, 1, x, n, out.as<double>(), part.as<double>(), kDotBlocks, E.stream);
  double v;
  d2h(&v, out.p, sizeof(double), E.stream);
  return std::sqrt(std::max(v, 0.0));
}

// ---------------------------------------------------------------------------
// MPS handling
// ---------------------------------------------------------------------------
void Engine::set_mps(int L_, const int* r, const double* const* Uh, const int32_t* const* q) {
  if (!have_mpo) throw std::logic_error("set the MPO before the TT iterate");
  if (L_ != L) throw std::invalid_argument("TT length differs from the MPO length");
  if (r[0] != 1 || r[L] != 1) throw std::invalid_argument("TT boundary ranks must be 1");
  std::vector<Labels> lab(L + 1);
  for (int k = 0; k <= L; ++k) {
    if (r[k] <= 0) throw std::invalid_argument("TT rank must be positive");
    lab[k].resize(r[k]);
    for (int a = 0; a < r[k]; ++a) lab[k][a] = {q[k][2 * a], q[k][2 * a + 1]};
  }
  if (lab[0][0] != Q2{0, 0}) throw std::invalid_argument("left boundary label must be (0,0)");
  std::vector<Core> cores(L);
  for (int k = 0; k < L; ++k) {
    Core& c = cores[k];
    c.rl = r[k]; c.rr = r[k + 1]; c.ql = lab[k]; c.qr = lab[k + 1];
    const int rlp = c.rlp(), rrp = c.rrp();
    std::vector<double> h((size_t)rlp * 4 * rrp, 0.0);
    for (int a = 0; a < c.rl; ++a)
      for (int s = 0; s < 4; ++s)
        for (int b = 0; b < c.rr; ++b) {
          double v = Uh[k][((size_t)a * 4 + s) * c.rr + b];
          if (v != 0.0 && qadd(c.ql[a], SITE_Q[s]) != c.qr[b])
            throw std::invalid_argument("TT core " + std::to_string(k) + " violates its quantum-number labels");
          h[((size_t)a * 4 + s) * rrp + b] = v;
        }
    upload(c.d, h.data(), h.size() * sizeof(double), stream);
  }
  for (int k = 0; k + 1 < L; ++k) qr_left(*this, cores[k], cores[k + 1]);
  double nrm = norm_dev(*this, cores[L - 1].d.as<double>(), cores[L - 1].elems());
  if (!(nrm > 0.0)) throw std::invalid_argument("TT iterate has zero norm");
  scale(cores[L - 1].d.as<double>(), 1.0 / nrm, cores[L - 1].elems(), stream);
  HC(hipStreamSynchronize(stream));
  U = std::move(cores);
  xscale = nrm;
  have_mps = true;
  free_caches();
}

// Right-hand side of the linear-system functional: kept as given (host layout checks as
// for the iterate).
void Engine::set_rhs(int L_, const int* r, const double* const* Fh, const int32_t* const* q) {
  if (!have_mpo) throw std::logic_error("set the MPO before the right-hand side");
  if (L_ != L) throw std::invalid_argument("right-hand side length differs from the MPO length");
  if (r[0] != 1 || r[L] != 1) throw std::invalid_argument("TT boundary ranks must be 1");
  std::vector<Labels> lab(L + 1);
  for (int k = 0; k <= L; ++k) {
    if (r[k] <= 0) throw std::invalid_argument("TT rank must be positive");
    lab[k].resize(r[k]);
    for (int a = 0; a < r[k]; ++a) lab[k][a] = {q[k][2 * a], q[k][2 * a + 1]};
  }
  if (lab[0][0] != Q2{0, 0}) throw std::invalid_argument("left boundary label must be (0,0)");
  std::vector<Core> cores(L);
  for (int k = 0; k < L; ++k) {
    Core& c = cores[k];
    c.rl = r[k]; c.rr = r[k + 1]; c.ql = lab[k]; c.qr = lab[k + 1];
    const int rlp = c.rlp(), rrp = c.rrp();
    std::vector<double> h((size_t)rlp * 4 * rrp, 0.0);
    for (int a = 0; a < c.rl; ++a)
      for (int s = 0; s < 4; ++s)
        for (int b = 0; b < c.rr; ++b) {
          double v = Fh[k][((size_t)a * 4 + s) * c.rr + b];
          if (v != 0.0 && qadd(c.ql[a], SITE_Q[s]) != c.qr[b])
            throw std::invalid_argument("right-hand side core " + std::to_string(k) + " violates its labels");
          h[((size_t)a * 4 + s) * rrp + b] = v;
        }
    upload(c.d, h.data(), h.size() * sizeof(double), stream);
  }
  HC(hipStreamSynchronize(stream));
  Fc = std::move(cores);
  have_rhs = true;
}

// E'[b'][b] = sum E[a'][a] bra[a'][s][b'] ket[a][s][b]  (dense, padded bonds)
void Engine::ov_left(const Env& in, const Core& bra, const Core& ket, Env& out) {
  if (in.R != 1 || in.rb != bra.rl || in.rk != ket.rl) throw std::runtime_error("ov_left: shape mismatch");
  const int rbp = padr(in.rb), rkp = padr(in.rk), rb2 = bra.rrp(), rk2 = ket.rrp();
  Env o;
  o.R = 1; o.rb = bra.rr; o.rk = ket.rr;
  o.d.ensure(sizeof(double) * o.elems());
  ws2.ensure(sizeof(double) * (size_t)rbp * 4 * rk2);
  GemmArgs g{};
  g.M = rbp; g.N = 4 * rk2; g.K = rkp; g.batch = 1; g.kin = rkp;
  g.sAm = rkp; g.sAkk = 1; g.sBkk = 4LL * rk2; g.sBn = 1; g.sCm = 4LL * rk2; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, in.d.as<double>(), ket.d.as<double>(), ws2.as<double>(), true, true, stream);
  GemmArgs h{};
  h.M = rb2; h.N = rk2; h.K = 4 * rbp; h.batch = 1; h.kin = 4 * rbp;
  h.sAm = 1; h.sAkk = rb2; h.sBkk = rk2; h.sBn = 1; h.sCm = rk2; h.alpha = 1.0; h.beta = 0.0;
  gemm<double>(h, bra.d.as<double>(), ws2.as<double>(), o.d.as<double>(), false, true, stream);
  out = std::move(o);
}

// E'[a'][a] = sum bra[a'][s][b'] ket[a][s][b] E[b'][b]  (dense, padded bonds)
void Engine::ov_right(const Env& in, const Core& bra, const Core& ket, Env& out) {
  if (in.R != 1 || in.rb != bra.rr || in.rk != ket.rr) throw std::runtime_error("ov_right: shape mismatch");
  const int rb2 = padr(in.rb), rk2 = padr(in.rk), rbp = bra.rlp(), rkp = ket.rlp();
  Env o;
  o.R = 1; o.rb = bra.rl; o.rk = ket.rl;
  o.d.ensure(sizeof(double) * o.elems());
  ws2.ensure(sizeof(double) * (size_t)rkp * 4 * rb2);
  GemmArgs g{};
  g.M = 4 * rkp; g.N = rb2; g.K = rk2; g.batch = 1; g.kin = rk2;
  g.sAm = rk2; g.sAkk = 1; g.sBkk = 1; g.sBn = rk2; g.sCm = rb2; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, ket.d.as<double>(), in.d.as<double>(), ws2.as<double>(), true, false, stream);
  GemmArgs h{};
  h.M = rbp; h.N = rkp; h.K = 4 * rb2; h.batch = 1; h.kin = 4 * rb2;
  h.sAm = 4LL * rb2; h.sAkk = 1; h.sBkk = 1; h.sBn = 4LL * rb2; h.sCm = rkp; h.alpha = 1.0; h.beta = 0.0;
  gemm<double>(h, bra.d.as<double>(), ws2.as<double>(), o.d.as<double>(), true, false, stream);
  out = std::move(o);
}

double Engine::overlap_with_rhs() {
  if (!have_rhs) throw std::logic_error("the linear-system functional needs tt_set_rhs");
  if (Fc.size() != (size_t)L || Fc[L - 1].qr != U[L - 1].qr)
    throw std::invalid_argument("right-hand side and iterate are in different sectors");
  Env e;
  env_unit(e, 1);
  for (int k = 0; k < L; ++k) {
    Env o;
    ov_left(e, U[k], Fc[k], o);
    e = std::move(o);
  }
  double v;
  d2h(&v, e.d.p, sizeof(double), stream);
  return v;
}

double Engine::functional_value() {
  if (opts.functional == 0) return energy();
  const double a = energy();  // <U|A|U>, U of unit norm
  return 0.5 * xscale * xscale * a - xscale * overlap_with_rhs();
}

void Engine::get_mps(int* r, double* const* Uh, int32_t* const* q) {
  if (!have_mps) throw std::logic_error("no TT iterate");
  r[0] = U[0].rl;
  for (int k = 0; k < L; ++k) r[k + 1] = U[k].rr;
  if (!Uh) return;
  for (int k = 0; k < L; ++k) {
    const Core& c = U[k];
    std::vector<double> h(c.elems());
    download(h.data(), c.d, h.size() * sizeof(double), stream);
    const int rrp = c.rrp();
    const double f = (opts.functional == 1 && k == L - 1) ? xscale : 1.0;
    for (int a = 0; a < c.rl; ++a)
      for (int s = 0; s < 4; ++s)
        for (int b = 0; b < c.rr; ++b) Uh[k][((size_t)a * 4 + s) * c.rr + b] = f * h[((size_t)a * 4 + s) * rrp + b];
  }
  if (q)
    for (int k = 0; k <= L; ++k) {
      const Labels& lab = k < L ? U[k].ql : U[L - 1].qr;
      for (size_t a = 0; a < lab.size(); ++a) {
        q[k][2 * a] = lab[a][0];
        q[k][2 * a + 1] = lab[a][1];
      }
    }
}

void Engine::checkpoint(int op) {
  auto copy = [&](const std::vector<Core>& from, std::vector<Core>& to) {
    to.clear();
    to.resize(from.size());
    for (size_t k = 0; k < from.size(); ++k) {
      Core& d = to[k];
      const Core& s = from[k];
      d.rl = s.rl; d.rr = s.rr; d.ql = s.ql; d.qr = s.qr;
      d.d.ensure(s.d.n);
      HC(hipMemcpyAsync(d.d.p, s.d.p, s.d.n, hipMemcpyDeviceToDevice, stream));
    }
    HC(hipStreamSynchronize(stream));
  };
  if (op == 0) {
    if (!have_mps) throw std::logic_error("checkpoint: no iterate to keep");
    copy(U, Usaved);
    xscale_saved = xscale;
  } else if (op == 1) {
    if (Usaved.empty()) throw std::logic_error("checkpoint: nothing kept");
    if ((int)Usaved.size() != L) throw std::logic_error("checkpoint: kept iterate does not fit the MPO");
    copy(Usaved, U);
    xscale = xscale_saved;
    free_caches();
    have_mps = true;
  } else {
    throw std::invalid_argument("checkpoint: op must be 0 (keep) or 1 (restore)");
  }
}

double Engine::energy() {
  if (!have_mps || !have_mpo) throw std::logic_error("energy needs MPO and TT");
  Env e;
  env_unit(e, 1);
  for (int k = 0; k < L; ++k) {
    Env o;
    env_left(e, U[k], U[k], k, o);
    e = std::move(o);
  }
  double v;
  d2h(&v, e.d.p, sizeof(double), stream);
  double n = norm_dev(*this, U[L - 1].d.as<double>(), U[L - 1].elems());
  return v / (n * n);
}

// ---------------------------------------------------------------------------
// local eigensolver (Davidson with FP64 Rayleigh-Ritz on the host)
// ---------------------------------------------------------------------------
struct Window {
  int rl = 0, rr = 0, rlp = 0, rrp = 0;
  int RA = 0, RAx = 0, RB = 0, RC = 0;
  const SiteOp* w1 = nullptr;
  const SiteOp* w2 = nullptr;
  DevMem Lx;            // FP64 left env incl. virtual channels [RAx][rlp][rlp]
  const double* R64 = nullptr;
  DevMem Rt;            // FP64 transformed right env [nP][rrp][rrp]
  int P0 = 0, nP = 0;
  int prec = 0;
  DevMem L32, R32, Rt32;  // low-precision copies
  DevMem diag;            // FP64 diagonal of the window operator [rlp][4][4][rrp]
  double flops = 0.0;
  bool use_tabs = false;
  WinTabs tabs;           // structural-zero tables of the quantum-number blocks (dense product)
  bool use_bs = false;
  BsPlan bs;              // block-sparse product plan
  int nphys = 16;         // local states of the window: 16 (two sites) or 4 (one site)
  bool one = false;       // one-site window (FP64 block-sparse product bs1, L in Lx, R in R64)
  BsHeff1 bs1;
  // HIP graphs of the block-sparse product's launches (tt_opts.graph_products), one per
  // product precision: captured at the second product with the same x and y, replayed
  // while they stay
  hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
  const double* gx[3] = {nullptr, nullptr, nullptr};
  double* gy[3] = {nullptr, nullptr, nullptr};
  // the engine workspaces a captured graph addresses (checked before every replay), the
  // precision the window's products have used, and whether graphs are off for it
  std::array<const void*, 16> gsig[3] = {};
  int gprec_used = -1;
  bool graph_off = false;
  Window() = default;
  Window(const Window&) = delete;
  Window& operator=(const Window&) = delete;
  ~Window() {
    for (hipGraphExec_t g : gexec)
      if (g) (void)hipGraphExecDestroy(g);
  }
};

// diag[a][s1][s2][b] = sum_B (sum_A W1[A,s1,s1,B] L_A[a][a]) (sum_C W2[B,s2,s2,C] R_C[b][b])
static void window_diag(Engine& E, Window& w, const Env& Le, int b, const Env& Re) {
  const SiteMPO& s1 = E.mpo[b];
  const SiteMPO& s2 = E.mpo[b + 1];
  DevMem Ld, Rd, LW, WR;
  Ld.ensure(sizeof(double) * (size_t)s1.Rl * w.rlp);
  Rd.ensure(sizeof(double) * (size_t)s2.Rr * w.rrp);
  LW.ensure(sizeof(double) * (size_t)s1.Rr * 4 * w.rlp);
  WR.ensure(sizeof(double) * (size_t)s1.Rr * 4 * w.rrp);
  diag_extract(Le.d.as<double>(), s1.Rl, w.rlp, Ld.as<double>(), E.stream);
  diag_extract(Re.d.as<double>(), s2.Rr, w.rrp, Rd.as<double>(), E.stream);
  diag_mix(s1.Rr, s1.byB.ptr.as<int>(), s1.byB.src.as<int>(), s1.byB.op64.as<double>(), Ld.as<double>(), w.rlp,
           LW.as<double>(), true, E.stream);
  diag_mix(s2.Rl, s2.byA.ptr.as<int>(), s2.byA.src.as<int>(), s2.byA.op64.as<double>(), Rd.as<double>(), w.rrp,
           WR.as<double>(), false, E.stream);
  w.diag.ensure(sizeof(double) * (size_t)w.rlp * 16 * w.rrp);
  GemmArgs g{};
  g.M = 4 * w.rlp; g.N = 4 * w.rrp; g.K = s1.Rr; g.batch = 1; g.kin = kin16(s1.Rr);
  g.sAm = 1; g.sAkk = 4LL * w.rlp; g.sBkk = 4LL * w.rrp; g.sBn = 1; g.sCm = 4LL * w.rrp; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, LW.as<double>(), WR.as<double>(), w.diag.as<double>(), false, true, E.stream);
  HC(hipStreamSynchronize(E.stream));
}

// ---------------------------------------------------------------------------
// structural zeros of the quantum-number blocks (tables read by the GEMM and
// mix kernels; every skipped product term is an exact zero)
// ---------------------------------------------------------------------------

// first and one-past-last index of every charge of a label list
static std::map<Q2, std::pair<int, int>> qspans(const Labels& q) {
  std::map<Q2, std::pair<int, int>> m;
  for (int i = 0; i < (int)q.size(); ++i) {
    auto it = m.find(q[i]);
    if (it == m.end()) m[q[i]] = {i, i + 1};
    else it->second.second = i + 1;
  }
  return m;
}

// distinct charges of the valid labels inside each tile of T consecutive indices
static std::vector<std::set<Q2>> tile_charges(const std::vector<Q2>& q, const std::vector<char>& valid, int n, int T) {
  const int nt = (n + T - 1) / T;
  std::vector<std::set<Q2>> out(nt);
  for (int i = 0; i < n; ++i)
    if (valid[i]) out[i / T].insert(q[i]);
  return out;
}

// K-range table of a batched product C_A = E_A X where E_A[m][k] can be non-zero
// only if q_m(m) - q_k(k) = d_A (kmode 1), plus the zero-tile map from the charges
// that X's columns need of k (colk[nt]).
static void kmode1_tables(const Labels& qm, int M, const Labels& qk, const std::vector<Q2>& dA,
                          const std::vector<std::set<Q2>>& colk, std::vector<int>& ktab, std::vector<uint8_t>& skip,
                          int& mtiles) {
  std::vector<Q2> qmv(M, Q2{QSENT, 0});
  std::vector<char> val(M, 0);
  for (int i = 0; i < (int)qm.size() && i < M; ++i) { qmv[i] = qm[i]; val[i] = 1; }
  const auto rowq = tile_charges(qmv, val, M, GEMM_TILE);
  mtiles = (int)rowq.size();
  const int ntiles = (int)colk.size();
  const auto spans = qspans(qk);
  const int nb = (int)dA.size();
  ktab.assign((size_t)nb * mtiles * 2, 0);
  skip.assign((size_t)nb * mtiles * ntiles, 1);
  std::map<Q2, int> seen;  // batches with equal channel charge share their rows
  for (int A = 0; A < nb; ++A) {
    auto it = seen.find(dA[A]);
    if (it != seen.end()) {
      const int B0 = it->second;
      std::copy(ktab.begin() + (size_t)B0 * mtiles * 2, ktab.begin() + (size_t)(B0 + 1) * mtiles * 2,
                ktab.begin() + (size_t)A * mtiles * 2);
      std::copy(skip.begin() + (size_t)B0 * mtiles * ntiles, skip.begin() + (size_t)(B0 + 1) * mtiles * ntiles,
                skip.begin() + (size_t)A * mtiles * ntiles);
      continue;
    }
    seen[dA[A]] = A;
    for (int mt = 0; mt < mtiles; ++mt) {
      std::set<Q2> need;  // charges of k that meet some row of the tile
      int lo = INT32_MAX, hi = 0;
      for (const Q2& r : rowq[mt]) {
        Q2 c = qsub(r, dA[A]);
        auto s = spans.find(c);
        if (s == spans.end()) continue;
        need.insert(c);
        lo = std::min(lo, s->second.first);
        hi = std::max(hi, s->second.second);
      }
      if (need.empty()) lo = hi = 0;
      ktab[((size_t)A * mtiles + mt) * 2] = lo;
      ktab[((size_t)A * mtiles + mt) * 2 + 1] = hi;
      for (int nt = 0; nt < ntiles; ++nt) {
        bool live = false;
        for (const Q2& c : need)
          if (colk[nt].count(c)) { live = true; break; }
        skip[((size_t)A * mtiles + mt) * ntiles + nt] = live ? 0 : 1;
      }
    }
  }
}

// inner K-range table of y = sum_C T_C R_C^T with R_C[n][k] non-zero only if
// q_n(n) - q_k(k) = d_C (kmode 2): ktab[(nt*nC + C)*2]
static void kmode2_tables(const Labels& qn, int N, const Labels& qk, const std::vector<Q2>& dC, std::vector<int>& ktab,
                          int& ntiles) {
  std::vector<Q2> qv(N, Q2{QSENT, 0});
  std::vector<char> val(N, 0);
  for (int i = 0; i < (int)qn.size() && i < N; ++i) { qv[i] = qn[i]; val[i] = 1; }
  const auto colq = tile_charges(qv, val, N, GEMM_TILE);
  ntiles = (int)colq.size();
  const auto spans = qspans(qk);
  const int nC = (int)dC.size();
  ktab.assign((size_t)ntiles * nC * 2, 0);
  std::map<Q2, std::vector<std::pair<int, int>>> memo;
  for (int C = 0; C < nC; ++C) {
    auto it = memo.find(dC[C]);
    if (it == memo.end()) {
      std::vector<std::pair<int, int>> r(ntiles, {0, 0});
      for (int nt = 0; nt < ntiles; ++nt) {
        int lo = INT32_MAX, hi = 0;
        for (const Q2& q : colq[nt]) {
          auto s = spans.find(qsub(q, dC[C]));
          if (s == spans.end()) continue;
          lo = std::min(lo, s->second.first);
          hi = std::max(hi, s->second.second);
        }
        if (hi == 0) lo = 0;
        r[nt] = {lo, hi};
      }
      it = memo.emplace(dC[C], std::move(r)).first;
    }
    for (int nt = 0; nt < ntiles; ++nt) {
      ktab[((size_t)nt * nC + C) * 2] = it->second[nt].first;
      ktab[((size_t)nt * nC + C) * 2 + 1] = it->second[nt].second;
    }
  }
}

// Tables of the two-site product at sites (b, b+1) with left labels ql (bond b)
// and right labels qr (bond b+2).
static void build_window_tabs(Engine& E, WinTabs& t, int b, const Labels& ql, const Labels& qr, int rlp, int rrp,
                              int RAx, int P0, int nP) {
  const SiteMPO& s1 = E.mpo[b];
  const SiteMPO& s2 = E.mpo[b + 1];
  // stage 1: T1[A] = L_A x over the left bond; channel A (or the virtual channel of
  // block row q) carries charge d_A with q(a') - q(a) = d_A
  std::vector<Q2> dA(RAx);
  for (int A = 0; A < s1.Rl; ++A) dA[A] = E.chan_q[b][A];
  for (int A = s1.Rl; A < RAx; ++A) dA[A] = E.chan_q[b + 1][s1.q0 + (A - s1.Rl)];
  // columns (s1, s2, b) of x need q(a) = q(b) - q(s1) - q(s2)
  const int N1 = 16 * rrp;
  std::vector<Q2> colq(N1, Q2{QSENT, 0});
  std::vector<char> colv(N1, 0);
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v)
      for (int j = 0; j < (int)qr.size(); ++j) {
        const int n = (u * 4 + v) * rrp + j;
        colq[n] = qsub(qsub(qr[j], SITE_Q[u]), SITE_Q[v]);
        colv[n] = 1;
      }
  const auto colk = tile_charges(colq, colv, N1, GEMM_TILE);
  t.n1tiles = (int)colk.size();
  std::vector<int> k1;
  std::vector<uint8_t> sk;
  kmode1_tables(ql, rlp, ql, dA, colk, k1, sk, t.m1tiles);
  upload(t.k1tab, k1.data(), k1.size() * sizeof(int), E.stream);
  upload(t.k1skip, sk.data(), sk.size(), E.stream);
  // stage 4: y = sum_C T3[C] R_C^T, R_C[b'][b] non-zero only if q(b') - q(b) = d_C
  std::vector<Q2> dC(E.chan_q[b + 2].begin(), E.chan_q[b + 2].end());
  std::vector<int> k4;
  kmode2_tables(qr, rrp, qr, dC, k4, t.n4tiles);
  upload(t.k4tab, k4.data(), k4.size() * sizeof(int), E.stream);
  if (nP > 0) {
    std::vector<Q2> dP(E.chan_q[b + 1].begin() + P0, E.chan_q[b + 1].begin() + P0 + nP);
    std::vector<int> kp;
    int nt = 0;
    kmode2_tables(qr, rrp, qr, dP, kp, nt);
    upload(t.k4tabP, kp.data(), kp.size() * sizeof(int), E.stream);
  }
  // mix charges: site 1 (O = a', I = (s2, b)), site 2 (O = (a', s1'), I = b)
  upload_q2(t.qo1, padded_q(ql, rlp, 1), E.stream);
  std::vector<Q2> qi1(4 * rrp, Q2{-QSENT, 0});
  for (int v = 0; v < 4; ++v)
    for (int j = 0; j < (int)qr.size(); ++j) qi1[v * rrp + j] = qsub(qr[j], SITE_Q[v]);
  upload_q2(t.qi1, qi1, E.stream);
  std::vector<Q2> qo2(4 * rlp, Q2{QSENT, 0});
  for (int a = 0; a < (int)ql.size(); ++a)
    for (int u = 0; u < 4; ++u) qo2[a * 4 + u] = qadd(ql[a], SITE_Q[u]);
  upload_q2(t.qo2, qo2, E.stream);
  upload_q2(t.qi2, padded_q(qr, rrp, -1), E.stream);
  t.qcB = E.chan_q_dev[b + 1].as<int2>();
  t.qcC = E.chan_q_dev[b + 2].as<int2>();
  (void)s2;
}

static void prepare_window(Engine& E, Window& w, const Env& Le, int b, const Env& Re, int prec, const Labels& ql,
                           const Labels& qr) {
  const SiteMPO& s1 = E.mpo[b];
  const SiteMPO& s2 = E.mpo[b + 1];
  w.rl = Le.rb; w.rr = Re.rb;
  w.rlp = padr(w.rl); w.rrp = padr(w.rr);
  w.RA = s1.Rl; w.RB = s1.Rr; w.RC = s2.Rr;
  const long long sl = (long long)w.rlp * w.rlp, sr = (long long)w.rrp * w.rrp;
  if (s1.has_block) {
    const int nQ = s1.q1 - s1.q0;
    w.RAx = w.RA + nQ;
    w.Lx.ensure(sizeof(double) * sl * w.RAx);
    HC(hipMemcpyAsync(w.Lx.p, Le.d.p, sizeof(double) * sl * w.RA, hipMemcpyDeviceToDevice, E.stream));
    channel_transform_qn(E, s1, Le.d.as<double>() + (long long)s1.p0 * sl, sl, w.Lx.as<double>() + (long long)w.RA * sl,
                         nQ, ql, ql, w.rlp, false);
    w.w1 = &s1.byB_left;
  } else {
    w.RAx = w.RA;
    w.Lx.ensure(sizeof(double) * sl * w.RA);
    HC(hipMemcpyAsync(w.Lx.p, Le.d.p, sizeof(double) * sl * w.RA, hipMemcpyDeviceToDevice, E.stream));
    w.w1 = &s1.byB;
  }
  w.R64 = Re.d.as<double>();
  if (s2.has_block) {
    w.P0 = s2.p0;
    w.nP = s2.p1 - s2.p0;
    w.Rt.ensure(sizeof(double) * sr * w.nP);
    channel_transform_qn(E, s2, Re.d.as<double>() + (long long)s2.q0 * sr, sr, w.Rt.as<double>(), w.nP, qr, qr, w.rrp,
                         true);
    w.w2 = &s2.byB_noblk;
  } else {
    w.nP = 0;
    w.w2 = &s2.byB;
  }
  w.prec = prec;
  w.use_bs = E.opts.qn_skip != 0 && bs_build(E, w.bs, b, ql, qr, w.rlp, w.rrp, w.RAx, w.nP);
  w.use_tabs = E.opts.qn_skip != 0 && !w.use_bs;
  if (w.use_bs && w.bs.lw)
    bs_lw_build(E, w.bs, w.Lx.as<double>(), sl * w.RAx, w.R64, w.nP ? w.Rt.as<double>() : nullptr);
  if (w.use_bs && w.bs.wr) {
    // with both operators precontracted the products read only LW and WR: the window's
    // copies of the environments were needed to form them, and no low-precision copies are
    // made (the diagonal preconditioner reads the environments themselves)
    w.Lx.release();
    w.Rt.release();
  } else if (prec == TT_BF16 && w.use_bs) {
    // block-sparse product in FP32 arithmetic on operands rounded to bfloat16
    w.L32.ensure(sizeof(float) * sl * w.RAx);
    convert_f64_bf16f32(w.Lx.as<double>(), w.L32.as<float>(), sl * w.RAx, E.stream);
    w.R32.ensure(sizeof(float) * sr * w.RC);
    convert_f64_bf16f32(w.R64, w.R32.as<float>(), sr * w.RC, E.stream);
    if (w.nP) {
      w.Rt32.ensure(sizeof(float) * sr * w.nP);
      convert_f64_bf16f32(w.Rt.as<double>(), w.Rt32.as<float>(), sr * w.nP, E.stream);
    }
  } else if (prec == TT_F32) {
    w.L32.ensure(sizeof(float) * sl * w.RAx);
    convert_f64_f32(w.Lx.as<double>(), w.L32.as<float>(), sl * w.RAx, E.stream);
    w.R32.ensure(sizeof(float) * sr * w.RC);
    convert_f64_f32(w.R64, w.R32.as<float>(), sr * w.RC, E.stream);
    if (w.nP) {
      w.Rt32.ensure(sizeof(float) * sr * w.nP);
      convert_f64_f32(w.Rt.as<double>(), w.Rt32.as<float>(), sr * w.nP, E.stream);
    }
  } else if (prec == TT_BF16) {
    w.L32.ensure(sizeof(uint16_t) * sl * w.RAx);
    convert_f64_bf16(w.Lx.as<double>(), w.L32.as<uint16_t>(), sl * w.RAx, E.stream);
    w.R32.ensure(sizeof(uint16_t) * sr * w.RC);
    convert_f64_bf16(w.R64, w.R32.as<uint16_t>(), sr * w.RC, E.stream);
    if (w.nP) {
      w.Rt32.ensure(sizeof(uint16_t) * sr * w.nP);
      convert_f64_bf16(w.Rt.as<double>(), w.Rt32.as<uint16_t>(), sr * w.nP, E.stream);
    }
  }
  // dense-bond algorithmic flops of one product (true sizes, no virtual channels)
  w.flops = 2.0 * 16.0 * w.rl * w.rr * ((double)w.RA * w.rl + (double)w.RC * w.rr);
  if (w.use_tabs) build_window_tabs(E, w.tabs, b, ql, qr, w.rlp, w.rrp, w.RAx, w.P0, w.nP);
  window_diag(E, w, Le, b, Re);
}

// the launches of one block-sparse two-site product (no host synchronisation)
static void bs_launch(Engine& E, Window& w, const double* x, double* y, int prec) {
  const size_t n = (size_t)w.rlp * 16 * w.rrp;
  if (prec == TT_F64) {
    bs_apply<double>(E, w.bs, w.Lx.as<double>(), w.R64, w.nP ? w.Rt.as<double>() : nullptr, x, y, false, false);
  } else {
    E.wlow_x.ensure(sizeof(float) * n);
    E.wlow_y.ensure(sizeof(float) * n);
    if (prec == TT_BF16) convert_f64_bf16f32(x, E.wlow_x.as<float>(), n, E.stream);
    else convert_f64_f32(x, E.wlow_x.as<float>(), n, E.stream);
    bs_apply<float>(E, w.bs, w.L32.as<float>(), w.R32.as<float>(), w.nP ? w.Rt32.as<float>() : nullptr,
                    E.wlow_x.as<float>(), E.wlow_y.as<float>(), prec == TT_BF16, false);
    convert_f32_f64(E.wlow_y.as<float>(), y, n, E.stream);
  }
}

// Block-sparse product through a HIP graph: the first product with (x, y, prec) runs
// eagerly (it makes the plan's one-time uploads and fills), the second is captured and
// every later one replays the captured launches.  Returns false when the product was not
// launched here (capture not possible): the caller then launches it eagerly.
static std::array<const void*, 16> bs_workspace_sig(const Engine& E) {
  std::array<const void*, 16> s{};
  int i = 0;
  for (const DevMem* m : {&E.bs_t1, &E.bs_t2, &E.bs_t3, &E.bs_part, &E.bs_tmp, &E.wlow_x, &E.wlow_y, &E.bs_x16})
    s[i++] = m->p;
  for (int b = 0; b < 4; ++b) {
    s[i++] = E.bs_gg1[b].p;
    s[i++] = E.bs_gg2[b].p;
  }
  return s;
}

// A graph replays launches whose operands include engine workspaces (intermediates, the
// heavy-row GEMM descriptors, T1's never-written entries, which an eager product zeroes
// when the precision changes).  Products of another precision on the same engine rewrite
// or reallocate them, so graphs are used only while a window's products keep one
// precision (the FP64-anchored refinement alternates: its windows run eagerly) and only
// while the workspaces are where they were at capture.
static bool bs_graph_product(Engine& E, Window& w, const double* x, double* y, int prec) {
  if (prec < 0 || prec > 2 || w.graph_off) return false;
  if (w.gprec_used >= 0 && w.gprec_used != prec) {
    for (hipGraphExec_t& g : w.gexec)
      if (g) {
        HC(hipGraphExecDestroy(g));
        g = nullptr;
      }
    w.graph_off = true;
    return false;
  }
  w.gprec_used = prec;
  hipGraphExec_t& ge = w.gexec[prec];
  if (ge && (w.gx[prec] != x || w.gy[prec] != y || w.gsig[prec] != bs_workspace_sig(E))) {
    HC(hipGraphExecDestroy(ge));
    ge = nullptr;
    w.gx[prec] = nullptr;  // the next product runs eagerly, the one after is captured
  }
  if (!ge) {
    const bool second = w.gx[prec] == x && w.gy[prec] == y;
    w.gx[prec] = x;
    w.gy[prec] = y;
    if (!second) return false;
    hipGraph_t g = nullptr;
    HC(hipStreamBeginCapture(E.stream, hipStreamCaptureModeThreadLocal));
    bool ok = true;
    try {
      bs_launch(E, w, x, y, prec);
    } catch (...) {
      ok = false;
    }
    const hipError_t ec = hipStreamEndCapture(E.stream, &g);
    if (ok && ec == hipSuccess && g && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) ge = nullptr;
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (!ge) return false;
    w.gsig[prec] = bs_workspace_sig(E);
  }
  HC(hipGraphLaunch(ge, E.stream));
  return true;
}

static void window_matvec(Engine& E, Window& w, const double* x, double* y, int prec) {
  const size_t n = (size_t)w.rlp * 16 * w.rrp;
  E.cur_rl = w.rl; E.cur_rr = w.rr; E.cur_RA = w.RA; E.cur_RC = w.RC;
  const WinTabs* tabs = w.use_tabs ? &w.tabs : nullptr;
  HC(hipEventRecord(E.ev0, E.stream));
  if (w.one) {
    if (prec != TT_F64) throw std::logic_error("one-site products run in FP64 only");
    bs_heff1_apply(E, w.bs1, w.Lx.as<double>(), x, y);
  } else if (w.use_bs) {
    // kernel timing records events between the launches: always eager
    const bool graphed = E.opts.graph_products && !E.kt_on && bs_graph_product(E, w, x, y, prec);
    if (!graphed) bs_launch(E, w, x, y, prec);
    bs_check(E, w.bs);
  } else if (prec == TT_F64) {
    E.heff<double>(w.rlp, w.rrp, w.RAx, w.Lx.as<double>(), *w.w1, w.RB, *w.w2, w.RC, w.R64, x, y,
                   w.nP ? w.Rt.as<double>() : nullptr, w.P0, w.nP, tabs);
  } else if (prec == TT_F32) {
    E.wlow_x.ensure(sizeof(float) * n);
    E.wlow_y.ensure(sizeof(float) * n);
    convert_f64_f32(x, E.wlow_x.as<float>(), n, E.stream);
    E.heff<float>(w.rlp, w.rrp, w.RAx, w.L32.as<float>(), *w.w1, w.RB, *w.w2, w.RC, w.R32.as<float>(),
                  E.wlow_x.as<float>(), E.wlow_y.as<float>(), w.nP ? w.Rt32.as<float>() : nullptr, w.P0, w.nP, tabs);
    convert_f32_f64(E.wlow_y.as<float>(), y, n, E.stream);
  } else {
    E.wlow_x.ensure(sizeof(uint16_t) * n);
    E.wlow_y.ensure(sizeof(float) * n);
    convert_f64_bf16(x, E.wlow_x.as<uint16_t>(), n, E.stream);
    E.heff_bf16(w.rlp, w.rrp, w.RAx, w.L32.as<uint16_t>(), *w.w1, w.RB, *w.w2, w.RC, w.R32.as<uint16_t>(),
                E.wlow_x.as<uint16_t>(), E.wlow_y.as<float>(), w.nP ? w.Rt32.as<uint16_t>() : nullptr, w.P0, w.nP,
                tabs);
    convert_f32_f64(E.wlow_y.as<float>(), y, n, E.stream);
  }
  HC(hipEventRecord(E.ev1, E.stream));
  HC(hipEventSynchronize(E.ev1));
  float ms = 0.f;
  HC(hipEventElapsedTime(&ms, E.ev0, E.ev1));
  E.sec_heff += ms * 1e-3;
  E.flops_heff += w.flops;
}

// The quantum-number-allowed entries of a two-site tensor (q(a) + q(s1) + q(s2) = q(b)):
// their positions in the padded dense layout [rlp][4][4][rrp], nc of them.  The local
// eigensolver keeps its vectors compressed to these entries, ncp = nc rounded up to 256
// long with a zero tail; a product expands its input into a dense tensor whose other
// entries stay zero and compresses its output, which also discards the output's
// entries outside the allowed ones.
struct QnIndex {
  DevMem idx;  // int32 [nc]
  size_t nc = 0, ncp = 0;
};
static QnIndex build_index(Engine& E, int rl, const Labels& ql, int rr, const Labels& qr) {
  const int rrp = padr(rr);
  std::vector<int> idx;
  for (int a = 0; a < rl; ++a)
    for (int s1 = 0; s1 < 4; ++s1)
      for (int s2 = 0; s2 < 4; ++s2) {
        Q2 q = qadd(qadd(ql[a], SITE_Q[s1]), SITE_Q[s2]);
        for (int b = 0; b < rr; ++b)
          if (qr[b] == q) idx.push_back((int)((((size_t)a * 4 + s1) * 4 + s2) * rrp + b));
      }
  QnIndex r;
  r.nc = idx.size();
  r.ncp = std::max<size_t>(256, (r.nc + 255) / 256 * 256);
  if (idx.empty()) idx.push_back(0);
  upload(r.idx, idx.data(), idx.size() * sizeof(int), E.stream);
  return r;
}

// Davidson for the lowest eigenpair of the window operator restricted to the
// QN-allowed entries.  x is the warm start on entry and the eigenvector on exit.
// Stops when the residual of the unit Ritz vector is <= max(tol, rel_tol * |theta|); with
// stop_on_stall also when it has not dropped below 0.9 x its best value for 8 iterations
// (a low-precision product has reached its rounding floor).
//
// anchor: the refinement of a low-precision solution (the precision split of the local
// solve).  The first basis vector's product is an FP64 one and every later direction's is
// in `prec`.  The Rayleigh-Ritz coupling of the first vector with the others then only
// involves FP64 products, so the low-precision rounding enters the Ritz vector through
// the correction directions alone, in proportion to their (small) weights.  A cycle ends
// when the residual has fallen 1000 times below its value at the cycle's start, stalls,
// or the basis is full; the next cycle's basis is the Ritz vector, with a fresh FP64
// product, and the next two Ritz vectors as correction directions.  The exact residual
// of the first basis vector is the only convergence test.  Each cycle thus gains about
// three digits for one FP64 product.
//
// nroots > 1 (Extension One): the nroots lowest eigenpairs, all to tol; the basis grows
// by the preconditioned residual of the lowest unconverged one; roots 1.. are written
// (dense, unit) to *extra.
static Davidson davidson(Engine& E, Window& w, const QnIndex& qi, double* x, int prec, double tol, int maxiter,
                         double rel_tol = 0.0, bool stop_on_stall = false, bool anchor = false, int nroots = 1,
                         std::vector<DevMem>* extra = nullptr) {
  Davidson res;
  const size_t nd = (size_t)w.rlp * w.nphys * w.rrp;  // dense tensor
  const size_t n = qi.ncp;                        // compressed vectors
  const int* idx = qi.idx.as<int>();
  const int maxsub = std::max(4, std::min(E.opts.dav_maxsub, 64));
  E.dav_V.ensure(sizeof(double) * n * maxsub);
  E.dav_AV.ensure(sizeof(double) * n * maxsub);
  E.dav_t.ensure(sizeof(double) * n);
  E.dav_u.ensure(sizeof(double) * n);
  E.dav_Au.ensure(sizeof(double) * n);
  E.dav_c.ensure(sizeof(double) * 2 * maxsub);
  E.dav_xd.ensure(sizeof(double) * nd);
  E.dav_yd.ensure(sizeof(double) * nd);
  E.dav_dc.ensure(sizeof(double) * n);
  const int nblk = kDotBlocks;
  E.wsp.ensure(sizeof(double) * (size_t)nblk * maxsub);
  double* V = E.dav_V.as<double>();
  double* AV = E.dav_AV.as<double>();
  double* t = E.dav_t.as<double>();
  double* u = E.dav_u.as<double>();
  double* Au = E.dav_Au.as<double>();
  double* cdev = E.dav_c.as<double>();
  double* part = E.wsp.as<double>();
  double* xd = E.dav_xd.as<double>();
  double* yd = E.dav_yd.as<double>();
  double* dg = E.dav_dc.as<double>();
  auto dots = [&](const double* Vb, int m, const double* vec, std::vector<double>& out) {
    multi_dot(Vb, n, m, vec, n, cdev, part, nblk, E.stream);
    out.resize(m);
    d2h(out.data(), cdev, sizeof(double) * m, E.stream);
  };
  auto lcomb = [&](const double* Vb, int m, const std::vector<double>& c, double* out) {
    HC(hipMemcpyAsync(cdev, c.data(), sizeof(double) * m, hipMemcpyHostToDevice, E.stream));
    lincomb(Vb, n, m, cdev, out, n, E.stream);
  };
  auto product = [&](const double* v, double* av, int p) {
    scatter_idx(xd, v, idx, qi.nc, E.stream);   // the other entries of xd stay zero
    window_matvec(E, w, xd, yd, p);
    gather_idx(av, yd, idx, qi.nc, n, E.stream);
    res.matvecs++;
    if (p == TT_F64) res.matvecs64++;
  };
  fill(xd, sizeof(double) * nd, E.stream);
  gather_idx(dg, w.diag.as<double>(), idx, qi.nc, n, E.stream);
  // start vector
  gather_idx(V, x, idx, qi.nc, n, E.stream);
  double nx = norm_dev(E, V, n);
  if (!(nx > 0.0)) {
    // fall back to a deterministic QN-allowed start: all allowed entries equal
    if (qi.nc == 0) throw std::runtime_error("empty QN-allowed space in a local problem");
    std::vector<double> h(n, 0.0);
    std::fill(h.begin(), h.begin() + qi.nc, 1.0);
    HC(hipMemcpyAsync(V, h.data(), sizeof(double) * n, hipMemcpyHostToDevice, E.stream));
    nx = norm_dev(E, V, n);
  }
  scale(V, 1.0 / nx, n, E.stream);
  product(V, AV, anchor ? TT_F64 : prec);
  int m = 1;
  std::vector<double> Hs((size_t)maxsub * maxsub, 0.0);
  {
    std::vector<double> d;
    dots(V, 1, AV, d);
    Hs[0] = d[0];
  }
  std::vector<double> evals, evecs, c;
  // anchored refinement: the next cycle's basis is the unit Ritz vector u, whose product
  // is taken again in FP64, and the next `more` Ritz vectors of the current basis with
  // their products combined from the stored ones (correction directions, orthogonal to
  // u); their couplings with u come from u's FP64 product
  auto anchor_restart = [&](int more) {
    more = std::max(0, std::min(more, m - 1));
    if (more) {
      E.dav_t2.ensure(sizeof(double) * n * more);
      E.dav_t3.ensure(sizeof(double) * n * more);
      for (int q = 0; q < more; ++q) {
        std::vector<double> cq(m);
        for (int i = 0; i < m; ++i) cq[i] = evecs[(size_t)i * m + q + 1];
        lcomb(V, m, cq, E.dav_t2.as<double>() + (size_t)q * n);
        lcomb(AV, m, cq, E.dav_t3.as<double>() + (size_t)q * n);
      }
    }
    std::vector<double> ev(evals.begin(), evals.end());
    double nu = norm_dev(E, u, n);
    HC(hipMemcpyAsync(V, u, sizeof(double) * n, hipMemcpyDeviceToDevice, E.stream));
    scale(V, 1.0 / nu, n, E.stream);
    if (more) {
      HC(hipMemcpyAsync(V + n, E.dav_t2.p, sizeof(double) * n * more, hipMemcpyDeviceToDevice, E.stream));
      HC(hipMemcpyAsync(AV + n, E.dav_t3.p, sizeof(double) * n * more, hipMemcpyDeviceToDevice, E.stream));
    }
    product(V, AV, TT_F64);
    std::vector<double> d;
    dots(V, 1 + more, AV, d);  // V_q . (A64 V_0)
    Hs.assign((size_t)maxsub * maxsub, 0.0);
    Hs[0] = d[0];
    for (int q = 1; q <= more; ++q) {
      Hs[(size_t)q * maxsub] = Hs[q] = d[q];
      Hs[(size_t)q * maxsub + q] = ev[q];
    }
    m = 1 + more;
  };
  double best = HUGE_VAL, cycle0 = HUGE_VAL;
  int since_best = 0;
  bool fresh = anchor;  // anchored: V_0's product is an FP64 one not yet checked
  for (int it = 0;; ++it) {
    if (fresh && m > 1) {
      // V_0 is the only basis vector whose product is entirely FP64: its residual is
      // exact, and it is the convergence test (the kept correction directions' products
      // are not)
      const double th0 = Hs[0];
      axpby(t, 1.0, AV, -th0, V, n, E.stream);
      const double r0 = norm_dev(E, t, n);
      if (r0 <= tol) {
        res.theta = th0;
        res.resid = r0;
        res.iters = it + 1;
        res.converged = true;
        HC(hipMemcpyAsync(u, V, sizeof(double) * n, hipMemcpyDeviceToDevice, E.stream));
        break;
      }
      cycle0 = r0;
    }
    // Rayleigh-Ritz
    std::vector<double> Hm((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Hm[(size_t)i * m + j] = 0.5 * (Hs[(size_t)i * maxsub + j] + Hs[(size_t)j * maxsub + i]);
    jacobi_eig(m, Hm, evals, evecs);
    res.theta = evals[0];
    c.resize(m);
    for (int i = 0; i < m; ++i) c[i] = evecs[(size_t)i * m];
    lcomb(V, m, c, u);
    lcomb(AV, m, c, Au);
    axpby(t, 1.0, Au, -res.theta, u, n, E.stream);
    res.resid = norm_dev(E, t, n);
    res.iters = it + 1;
    double theta_x = res.theta;  // the shift of the next direction's preconditioner
    bool roots_done = false;
    if (nroots > 1) {
      // residuals of the nroots lowest Ritz pairs; t becomes that of the lowest
      // unconverged one
      const int nr = std::min(nroots, m);
      E.dav_uk.ensure(sizeof(double) * n * nroots);
      E.dav_tk.ensure(sizeof(double) * n);
      double* tk = E.dav_tk.as<double>();
      int pick = res.resid > tol ? 0 : -1;
      double rmax = res.resid;
      HC(hipMemcpyAsync(E.dav_uk.p, u, sizeof(double) * n, hipMemcpyDeviceToDevice, E.stream));
      for (int q = 1; q < nr; ++q) {
        std::vector<double> cq(m);
        for (int i = 0; i < m; ++i) cq[i] = evecs[(size_t)i * m + q];
        double* uq = E.dav_uk.as<double>() + (size_t)q * n;
        lcomb(V, m, cq, uq);
        lcomb(AV, m, cq, tk);
        axpby(tk, 1.0, tk, -evals[q], uq, n, E.stream);
        const double rq = norm_dev(E, tk, n);
        rmax = std::max(rmax, rq);
        if (rq > tol && pick < 0) {
          pick = q;
          theta_x = evals[q];
          HC(hipMemcpyAsync(t, tk, sizeof(double) * n, hipMemcpyDeviceToDevice, E.stream));
        }
      }
      roots_done = nr == nroots && pick < 0;
      if (pick < 0 && nr < nroots) {
        // fewer basis vectors than roots, all of them converged: grow from the last one
        pick = nr - 1;
        theta_x = evals[pick];
        if (pick > 0) HC(hipMemcpyAsync(t, tk, sizeof(double) * n, hipMemcpyDeviceToDevice, E.stream));
      }
      res.resid = rmax;
    }
    if (anchor) {
      if (fresh) {
        fresh = false;
        if (m == 1) {
          // u = V_0: theta and the residual are exact
          if (res.resid <= tol) {
            res.converged = true;
            break;
          }
          cycle0 = res.resid;
        }
        best = res.resid;
        since_best = 0;
      } else {
        bool end_cycle = res.resid <= 1e-3 * cycle0 || res.resid <= 0.5 * tol || m >= maxsub;
        if (res.resid < 0.9 * best) {
          best = res.resid;
          since_best = 0;
        } else if (++since_best >= 6) {
          end_cycle = true;
        }
        if (end_cycle) {
          if (res.matvecs >= maxiter) break;
          anchor_restart(2);
          fresh = true;
          continue;
        }
      }
    } else {
      if (nroots > 1 ? roots_done : res.resid <= std::max(tol, rel_tol * std::fabs(res.theta))) {
        res.converged = true;
        break;
      }
      if (stop_on_stall) {
        if (res.resid < 0.9 * best) {
          best = res.resid;
          since_best = 0;
        } else if (++since_best >= 8) {
          break;
        }
      }
    }
    if (res.matvecs >= maxiter) break;
    if (m >= maxsub) {
      // thick restart: keep the lowest Ritz vectors of the current subspace
      const int keep = std::min(std::max(3, nroots + 2), m);
      E.dav_t2.ensure(sizeof(double) * n * keep);
      E.dav_t3.ensure(sizeof(double) * n * keep);
      for (int q = 0; q < keep; ++q) {
        std::vector<double> cq(m);
        for (int i = 0; i < m; ++i) cq[i] = evecs[(size_t)i * m + q];
        lcomb(V, m, cq, E.dav_t2.as<double>() + (size_t)q * n);
        lcomb(AV, m, cq, E.dav_t3.as<double>() + (size_t)q * n);
      }
      HC(hipMemcpyAsync(V, E.dav_t2.p, sizeof(double) * n * keep, hipMemcpyDeviceToDevice, E.stream));
      HC(hipMemcpyAsync(AV, E.dav_t3.p, sizeof(double) * n * keep, hipMemcpyDeviceToDevice, E.stream));
      Hs.assign((size_t)maxsub * maxsub, 0.0);
      for (int q = 0; q < keep; ++q) Hs[(size_t)q * maxsub + q] = evals[q];
      m = keep;
      continue;
    }
    // new direction: diagonally preconditioned residual, projected out of the subspace
    // (classical Gram-Schmidt, repeated once when the first pass cancels more than a
    // factor 1/sqrt(2) of the norm: "twice is enough")
    // The direction is formed in its basis slot V_m, so one multi-dot over V_0..V_m
    // gives the projections and the squared norm together.
    double* vm = V + (size_t)m * n;
    precond(vm, t, dg, theta_x, nullptr, n, E.stream);
    std::vector<double> d;
    dots(V, m + 1, vm, d);
    const double tn0 = std::sqrt(std::max(d[m], 0.0));
    double tn = tn0;
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<double> c(d.begin(), d.begin() + m);
      for (double& v : c) v = -v;
      // the residual t has been consumed by the preconditioner, so it holds the
      // projection; u stays the Ritz vector that theta and resid describe, which is
      // what every exit below returns
      lcomb(V, m, c, t);
      axpy(vm, 1.0, t, n, E.stream);
      dots(V, m + 1, vm, d);
      const double prev = tn;
      tn = std::sqrt(std::max(d[m], 0.0));
      if (tn >= prev / std::sqrt(2.0)) break;
    }
    if (!(tn > 1e-10 * tn0) || !(tn > 0.0)) {
      // the search space is exhausted
      if (anchor && m > 1 && res.matvecs < maxiter) {
        anchor_restart(0);  // confirm the Ritz vector with an exact residual
        fresh = true;
        continue;
      }
      res.converged = !anchor && res.resid <= tol;
      break;
    }
    scale(vm, 1.0 / tn, n, E.stream);
    double* avm = AV + (size_t)m * n;
    product(vm, avm, prec);
    dots(V, m + 1, avm, d);
    if (anchor) {
      // the coupling with the first basis vector from that vector's FP64 product
      std::vector<double> d0;
      dots(AV, 1, vm, d0);
      d[0] = d0[0];
    }
    for (int i = 0; i <= m; ++i) {
      Hs[(size_t)i * maxsub + m] = d[i];
      Hs[(size_t)m * maxsub + i] = d[i];
    }
    ++m;
  }
  // eigenvector -> x (unit norm, zero outside the allowed entries)
  double nu = norm_dev(E, u, n);
  scale(u, 1.0 / nu, n, E.stream);
  fill(x, sizeof(double) * nd, E.stream);
  scatter_idx(x, u, idx, qi.nc, E.stream);
  if (nroots > 1 && extra) {
    extra->resize(nroots - 1);
    for (int q = 1; q < nroots; ++q) {
      DevMem& X = (*extra)[q - 1];
      X.ensure(sizeof(double) * nd);
      fill(X.p, sizeof(double) * nd, E.stream);
      if (q < m) {
        double* uq = E.dav_uk.as<double>() + (size_t)q * n;
        const double nq = norm_dev(E, uq, n);
        scale(uq, 1.0 / nq, n, E.stream);
        scatter_idx(X.as<double>(), uq, idx, qi.nc, E.stream);
      }
    }
  }
  HC(hipStreamSynchronize(E.stream));
  return res;
}

// one micro-iteration: lowest eigenpair of the window; returns theta
// With more != nullptr and coarse_k > 1 (Extension One), the coarse_k lowest eigenpairs
// with FP64 products; roots 1.. go to *more (as many as the local space allows).
static Davidson local_eig(Engine& E, const Env& Le, int b, const Env& Re, DevMem& x, const Core& C, const Core& D,
                          std::vector<DevMem>* more = nullptr) {
  const Labels& ql = C.ql;
  const Labels& qr = D.qr;
  QnIndex mask = build_index(E, C.rl, ql, D.rr, qr);
  Window w;
  const int prec = E.opts.matvec_prec;
  Davidson r;
  double tph = E.now();
  if (more && E.opts.coarse_k > 1) {
    const int K = (int)std::min<size_t>(E.opts.coarse_k, mask.nc);
    prepare_window(E, w, Le, b, Re, TT_F64, ql, qr);
    E.ph[2] += E.now() - tph;
    tph = E.now();
    r = davidson(E, w, mask, x.as<double>(), TT_F64, E.opts.dav_tol, E.opts.dav_maxiter, 0.0, false, false, K, more);
    E.ph[3] += E.now() - tph;
    if (!r.converged) E.warn = std::max(E.warn, (int)TT_WNOCONV);
    return r;
  }
  if (prec != TT_F64) {
    prepare_window(E, w, Le, b, Re, prec, ql, qr);
    E.ph[2] += E.now() - tph;
    tph = E.now();
    if (E.opts.refine_fp64)
      r = davidson(E, w, mask, x.as<double>(), prec, E.opts.dav_tol, E.opts.dav_maxiter, E.opts.lowprec_tol, true);
    else
      r = davidson(E, w, mask, x.as<double>(), prec, E.opts.dav_tol, E.opts.dav_maxiter);
    if (E.opts.refine_fp64) {
      // refinement: FP64 residuals with FP32 correction directions.  A bfloat16 product
      // is too coarse for the corrections (its rounding error exceeds the gap-scaled
      // residual), so a block-sparse bfloat16 window is converted to FP32 operands (same
      // storage), and a dense bfloat16 window continues with FP64 products.
      int inner = prec;
      if (prec == TT_BF16) {
        if (w.use_bs && w.bs.wr) {
          inner = TT_F32;  // the FP32 copies of LW and WR follow the product precision
        } else if (w.use_bs) {
          const long long sl = (long long)w.rlp * w.rlp, sr = (long long)w.rrp * w.rrp;
          convert_f64_f32(w.Lx.as<double>(), w.L32.as<float>(), sl * w.RAx, E.stream);
          convert_f64_f32(w.R64, w.R32.as<float>(), sr * w.RC, E.stream);
          if (w.nP) convert_f64_f32(w.Rt.as<double>(), w.Rt32.as<float>(), sr * w.nP, E.stream);
          w.bs.have32 = false;  // the stacked right environment follows the new operands
          inner = TT_F32;
        } else {
          inner = -1;
        }
      }
      const int left = std::max(1, E.opts.dav_maxiter - r.matvecs);
      Davidson r2;
      if (inner >= 0) {
        r2 = davidson(E, w, mask, x.as<double>(), inner, E.opts.dav_tol, left, 0.0, false, true);
      } else {
        w.L32.release();
        w.R32.release();
        w.Rt32.release();
        r2 = davidson(E, w, mask, x.as<double>(), TT_F64, E.opts.dav_tol, left);
      }
      r2.matvecs += r.matvecs;
      r2.matvecs64 += r.matvecs64;
      r = r2;
    }
  } else {
    prepare_window(E, w, Le, b, Re, TT_F64, ql, qr);
    E.ph[2] += E.now() - tph;
    tph = E.now();
    r = davidson(E, w, mask, x.as<double>(), TT_F64, E.opts.dav_tol, E.opts.dav_maxiter);
  }
  E.ph[3] += E.now() - tph;
  if (!r.converged) E.warn = std::max(E.warn, (int)TT_WNOCONV);
  return r;
}

// ---------------------------------------------------------------------------
// linear-system functional: projected right-hand side and conjugate gradients
// ---------------------------------------------------------------------------

// P^T F of the window in its dense layout [rlp][nphys][rrp]: the overlap environments FLe
// ([1][rl][rFl]) and FRe ([1][rr][rFr]) with F's cores of the window (one or two) between.
static void local_rhs(Engine& E, const Window& w, const Env& FLe, const Env& FRe, const Core* F1, const Core* F2,
                      double* b) {
  const int rFl = F1->rlp(), rFr = (F2 ? F2 : F1)->rrp();
  const int np = w.nphys;
  if (FLe.rb != w.rl || FRe.rb != w.rr || FLe.rk != F1->rl || FRe.rk != (F2 ? F2 : F1)->rr)
    throw std::runtime_error("projected right-hand side: shape mismatch");
  DevMem T, Y1;
  const double* Ft = F1->d.as<double>();
  if (F2) {
    // F1 F2 -> [rFl][4][4][rFr]
    const int kp = F1->rrp();
    T.ensure(sizeof(double) * (size_t)rFl * 16 * rFr);
    GemmArgs g{};
    g.M = 4 * rFl; g.N = 4 * rFr; g.K = kp; g.batch = 1; g.kin = kp;
    g.sAm = kp; g.sAkk = 1; g.sBkk = 4LL * rFr; g.sBn = 1; g.sCm = 4LL * rFr; g.alpha = 1.0; g.beta = 0.0;
    gemm<double>(g, F1->d.as<double>(), F2->d.as<double>(), T.as<double>(), true, true, E.stream);
    Ft = T.as<double>();
  }
  // Y1[a][(s..)][bF] = sum_aF FL[a][aF] Ft[aF][(s..)][bF]
  Y1.ensure(sizeof(double) * (size_t)w.rlp * np * rFr);
  GemmArgs g{};
  g.M = w.rlp; g.N = np * rFr; g.K = rFl; g.batch = 1; g.kin = rFl;
  g.sAm = rFl; g.sAkk = 1; g.sBkk = (long long)np * rFr; g.sBn = 1; g.sCm = (long long)np * rFr;
  g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, FLe.d.as<double>(), Ft, Y1.as<double>(), true, true, E.stream);
  // b[(a s..)][b'] = sum_bF Y1[(a s..)][bF] FR[b'][bF]
  GemmArgs h{};
  h.M = w.rlp * np; h.N = w.rrp; h.K = rFr; h.batch = 1; h.kin = rFr;
  h.sAm = rFr; h.sAkk = 1; h.sBkk = 1; h.sBn = rFr; h.sCm = w.rrp; h.alpha = 1.0; h.beta = 0.0;
  gemm<double>(h, Y1.as<double>(), FRe.d.as<double>(), b, true, false, E.stream);
  HC(hipStreamSynchronize(E.stream));
}

// Micro-step of the linear-system functional: minimise 1/2 w.Aw - b.w over the allowed
// entries, i.e. solve P^T A P w = P^T F (A symmetric positive definite), by conjugate
// gradients preconditioned with the diagonal, from the warm start x, until the residual is
// <= tol |b|.  theta returns the local minimum 1/2 w.Aw - b.w = -(w.b + w.r)/2.
static Davidson pcg(Engine& E, Window& w, const QnIndex& qi, double* x, const double* bdense, double tol,
                    int maxiter) {
  Davidson res;
  const size_t nd = (size_t)w.rlp * w.nphys * w.rrp;
  const size_t n = qi.ncp;
  const int* idx = qi.idx.as<int>();
  E.dav_V.ensure(sizeof(double) * n * 4);
  E.dav_AV.ensure(sizeof(double) * n * 2);
  E.dav_xd.ensure(sizeof(double) * nd);
  E.dav_yd.ensure(sizeof(double) * nd);
  E.dav_dc.ensure(sizeof(double) * n);
  E.dav_c.ensure(sizeof(double) * 8);
  E.wsp.ensure(sizeof(double) * (size_t)kDotBlocks * 2);
  double* xc = E.dav_V.as<double>();
  double* r = xc + n;
  double* z = xc + 2 * n;
  double* pv = xc + 3 * n;
  double* q = E.dav_AV.as<double>();
  double* bc = q + n;
  double* xd = E.dav_xd.as<double>();
  double* yd = E.dav_yd.as<double>();
  double* dg = E.dav_dc.as<double>();
  double* cdev = E.dav_c.as<double>();
  double* part = E.wsp.as<double>();
  auto dot = [&](const double* a, const double* b2) {
    multi_dot(a, n, 1, b2, n, cdev, part, kDotBlocks, E.stream);
    double v;
    d2h(&v, cdev, sizeof(double), E.stream);
    return v;
  };
  auto product = [&](const double* v, double* av) {
    scatter_idx(xd, v, idx, qi.nc, E.stream);
    window_matvec(E, w, xd, yd, TT_F64);
    gather_idx(av, yd, idx, qi.nc, n, E.stream);
    res.matvecs++;
    res.matvecs64++;
  };
  // z = r / diag (the kernel returns r / (theta - d))
  auto prec = [&](const double* rv, double* zv) {
    precond(zv, rv, dg, 0.0, nullptr, n, E.stream);
    scale(zv, -1.0, n, E.stream);
  };
  fill(xd, sizeof(double) * nd, E.stream);
  gather_idx(dg, w.diag.as<double>(), idx, qi.nc, n, E.stream);
  gather_idx(bc, bdense, idx, qi.nc, n, E.stream);
  gather_idx(xc, x, idx, qi.nc, n, E.stream);
  const double bnorm = std::sqrt(std::max(dot(bc, bc), 0.0));
  if (!(bnorm > 0.0)) {
    // P^T F = 0: the minimiser is w = 0
    fill(x, sizeof(double) * nd, E.stream);
    res.converged = true;
    res.theta = 0.0;
    HC(hipStreamSynchronize(E.stream));
    return res;
  }
  product(xc, q);
  axpby(r, 1.0, bc, -1.0, q, n, E.stream);  // r = b - A x
  double rn = std::sqrt(std::max(dot(r, r), 0.0));
  prec(r, z);
  HC(hipMemcpyAsync(pv, z, sizeof(double) * n, hipMemcpyDeviceToDevice, E.stream));
  double rz = dot(r, z);
  while (rn > tol * bnorm && res.matvecs < maxiter) {
    product(pv, q);
    const double pq = dot(pv, q);
    if (!(pq > 0.0)) throw std::runtime_error("linear-system functional: the local operator is not positive definite");
    const double alpha = rz / pq;
    axpy(xc, alpha, pv, n, E.stream);
    axpy(r, -alpha, q, n, E.stream);
    rn = std::sqrt(std::max(dot(r, r), 0.0));
    ++res.iters;
    if (rn <= tol * bnorm) break;
    prec(r, z);
    const double rz2 = dot(r, z);
    axpby(pv, 1.0, z, rz2 / rz, pv, n, E.stream);  // p = z + beta p
    rz = rz2;
  }
  res.converged = rn <= tol * bnorm;
  res.resid = rn / bnorm;
  res.theta = -0.5 * (dot(xc, bc) + dot(xc, r));
  fill(x, sizeof(double) * nd, E.stream);
  scatter_idx(x, xc, idx, qi.nc, E.stream);
  HC(hipStreamSynchronize(E.stream));
  return res;
}

// Linear-system micro-step of the window at bond (b, b+1) (two-site: C, D the current
// cores) or at site b (one-site: C the current core, D unused); x the warm start.
static Davidson local_lin(Engine& E, const Env& Le, int b, const Env& Re, DevMem& x, const Core& C, const Core* D,
                          const Env& FLe, const Env& FRe, const Core& F1, const Core* F2);

// ---------------------------------------------------------------------------
// one-site local problems (Algorithm 2, one-site branch)
// ---------------------------------------------------------------------------

// The quantum-number-allowed entries q(a) + q(s) = q(b) of a core, in the padded
// layout [rlp][4][rrp] (as build_index for two-site tensors).
static QnIndex build_index1(Engine& E, int rl, const Labels& ql, int rr, const Labels& qr) {
  const int rrp = padr(rr);
  std::vector<int> idx;
  for (int a = 0; a < rl; ++a)
    for (int s = 0; s < 4; ++s) {
      const Q2 q = qadd(ql[a], SITE_Q[s]);
      for (int b = 0; b < rr; ++b)
        if (qr[b] == q) idx.push_back((int)(((size_t)a * 4 + s) * rrp + b));
    }
  QnIndex r;
  r.nc = idx.size();
  r.ncp = std::max<size_t>(256, (r.nc + 255) / 256 * 256);
  if (idx.empty()) idx.push_back(0);
  upload(r.idx, idx.data(), idx.size() * sizeof(int), E.stream);
  return r;
}

// diag[a][s][b] = sum_B (sum_A W[A,s,s,B] L_A[a][a]) R_B[b][b]
static void window_diag1(Engine& E, Window& w, const Env& Le, int k, const Env& Re) {
  const SiteMPO& sm = E.mpo[k];
  DevMem Ld, Rd, LW;
  Ld.ensure(sizeof(double) * (size_t)sm.Rl * w.rlp);
  Rd.ensure(sizeof(double) * (size_t)sm.Rr * w.rrp);
  LW.ensure(sizeof(double) * (size_t)sm.Rr * 4 * w.rlp);
  diag_extract(Le.d.as<double>(), sm.Rl, w.rlp, Ld.as<double>(), E.stream);
  diag_extract(Re.d.as<double>(), sm.Rr, w.rrp, Rd.as<double>(), E.stream);
  diag_mix(sm.Rr, sm.byB.ptr.as<int>(), sm.byB.src.as<int>(), sm.byB.op64.as<double>(), Ld.as<double>(), w.rlp,
           LW.as<double>(), true, E.stream);
  w.diag.ensure(sizeof(double) * (size_t)w.rlp * 4 * w.rrp);
  GemmArgs g{};
  g.M = 4 * w.rlp; g.N = w.rrp; g.K = sm.Rr; g.batch = 1; g.kin = kin16(sm.Rr);
  g.sAm = 1; g.sAkk = 4LL * w.rlp; g.sBkk = w.rrp; g.sBn = 1; g.sCm = w.rrp; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, LW.as<double>(), Rd.as<double>(), w.diag.as<double>(), false, true, E.stream);
  HC(hipStreamSynchronize(E.stream));
}

// One-site window of site k: Le at bond k, Re at bond k + 1 (FP64).
static void prepare_window1(Engine& E, Window& w, const Env& Le, int k, const Env& Re, const Labels& ql,
                            const Labels& qr) {
  const SiteMPO& sm = E.mpo[k];
  w.one = true;
  w.nphys = 4;
  w.rl = Le.rb; w.rr = Re.rb;
  w.rlp = padr(w.rl); w.rrp = padr(w.rr);
  if ((int)ql.size() != w.rl || (int)qr.size() != w.rr) throw std::runtime_error("one-site window: label mismatch");
  w.RA = sm.Rl; w.RB = sm.Rr; w.RC = sm.Rr;
  const long long sl = (long long)w.rlp * w.rlp;
  w.RAx = w.RA + (sm.has_block ? sm.q1 - sm.q0 : 0);
  w.Lx.ensure(sizeof(double) * sl * w.RAx);
  HC(hipMemcpyAsync(w.Lx.p, Le.d.p, sizeof(double) * sl * w.RA, hipMemcpyDeviceToDevice, E.stream));
  if (sm.has_block)
    channel_transform_qn(E, sm, Le.d.as<double>() + (long long)sm.p0 * sl, sl, w.Lx.as<double>() + (long long)w.RA * sl,
                         sm.q1 - sm.q0, ql, ql, w.rlp, false);
  w.R64 = Re.d.as<double>();
  w.prec = TT_F64;
  if (!bs_heff1_build(E, w.bs1, E.left_site_use(k), ql, qr, w.RAx, w.R64, w.RB))
    throw std::runtime_error("one-site product: bond labels are not grouped by charge");
  // dense-bond algorithmic flops of one product (both contractions, true sizes)
  w.flops = 2.0 * 4.0 * w.rl * w.rr * ((double)w.RA * w.rl + (double)w.RB * w.rr);
  window_diag1(E, w, Le, k, Re);
}

// one-site micro-iteration at site k: lowest eigenpair of the one-site window (FP64
// products), warm-started from x; with more != nullptr and coarse_k > 1 the coarse_k
// lowest (Extension One), roots 1.. into *more.
static Davidson local_eig1(Engine& E, const Env& Le, int k, const Env& Re, DevMem& x, const Core& C,
                           std::vector<DevMem>* more = nullptr) {
  QnIndex mask = build_index1(E, C.rl, C.ql, C.rr, C.qr);
  Window w;
  double tph = E.now();
  prepare_window1(E, w, Le, k, Re, C.ql, C.qr);
  E.ph[2] += E.now() - tph;
  tph = E.now();
  Davidson r;
  if (more && E.opts.coarse_k > 1) {
    const int K = (int)std::min<size_t>(E.opts.coarse_k, mask.nc);
    r = davidson(E, w, mask, x.as<double>(), TT_F64, E.opts.dav_tol, E.opts.dav_maxiter, 0.0, false, false, K, more);
  } else {
    r = davidson(E, w, mask, x.as<double>(), TT_F64, E.opts.dav_tol, E.opts.dav_maxiter);
  }
  E.ph[3] += E.now() - tph;
  if (!r.converged) E.warn = std::max(E.warn, (int)TT_WNOCONV);
  return r;
}

static Davidson local_lin(Engine& E, const Env& Le, int b, const Env& Re, DevMem& x, const Core& C, const Core* D,
                          const Env& FLe, const Env& FRe, const Core& F1, const Core* F2) {
  const bool one = D == nullptr;
  QnIndex mask = one ? build_index1(E, C.rl, C.ql, C.rr, C.qr) : build_index(E, C.rl, C.ql, D->rr, D->qr);
  Window w;
  double tph = E.now();
  if (one) prepare_window1(E, w, Le, b, Re, C.ql, C.qr);
  else prepare_window(E, w, Le, b, Re, TT_F64, C.ql, D->qr);
  DevMem bd;
  bd.ensure(sizeof(double) * (size_t)w.rlp * w.nphys * w.rrp);
  local_rhs(E, w, FLe, FRe, &F1, F2, bd.as<double>());
  E.ph[2] += E.now() - tph;
  tph = E.now();
  Davidson r = pcg(E, w, mask, x.as<double>(), bd.as<double>(), E.opts.dav_tol, E.opts.dav_maxiter);
  E.ph[3] += E.now() - tph;
  if (!r.converged) E.warn = std::max(E.warn, (int)TT_WNOCONV);
  return r;
}

// ---------------------------------------------------------------------------
// Step 1 + Step 2
// ---------------------------------------------------------------------------
void Engine::solve_subdomain(const Engine& src, int j, int s, int e, Sub& S) {
  double tph = 0.0;
  const int blast = std::min(e, L - 2);
  S = Sub();
  S.s = s;
  S.t = blast + 1;
  if (s > L - 2) {
    // a one-site last subdomain has no bond of its own
    S.t = s;
    S.mod.clear();
    Core c;
    c.rl = src.Wc[s].rl; c.rr = src.Wc[s].rr; c.ql = src.Wc[s].ql; c.qr = src.Wc[s].qr;
    c.d.ensure(src.Wc[s].d.n);
    HC(hipMemcpyAsync(c.d.p, src.Wc[s].d.p, src.Wc[s].d.n, hipMemcpyDeviceToDevice, stream));
    S.mod.push_back(std::move(c));
    S.E = 0.0;
    HC(hipStreamSynchronize(stream));
    return;
  }
  Core center;
  center.rl = src.Wc[s].rl; center.rr = src.Wc[s].rr; center.ql = src.Wc[s].ql; center.qr = src.Wc[s].qr;
  center.d.ensure(src.Wc[s].d.n);
  HC(hipMemcpyAsync(center.d.p, src.Wc[s].d.p, src.Wc[s].d.n, hipMemcpyDeviceToDevice, stream));
  Env Lrun;
  const Env* Lcur = &src.Lenv[s];
  // linear-system functional: the warm start carries the iterate's norm, and the overlap
  // environment with F moves along with Lrun
  const bool lin = opts.functional == 1;
  Env FLrun;
  const Env* FLcur = lin ? &src.FL[s] : nullptr;
  if (lin) scale(center.d.as<double>(), src.xscale, center.elems(), stream);
  DevMem x;
  for (int b = s; b <= blast; ++b) {
    const Core& next = src.Vc[b + 1];
    two_site(*this, center, next, x);
    std::vector<DevMem> more;
    Davidson r = lin ? local_lin(*this, *Lcur, b, src.Renv[b + 2], x, center, &next, *FLcur, src.FR[b + 2],
                                 src.Fc[b], &src.Fc[b + 1])
                     : local_eig(*this, *Lcur, b, src.Renv[b + 2], x, center, next,
                                 b == blast && opts.coarse_k > 1 ? &more : nullptr);
    S.matvecs += r.matvecs;
    S.matvecs64 += r.matvecs64;
    S.E = r.theta;
    S.converged = S.converged && r.converged;
    Core N, C;
    tph = now();
    split_two_site(*this, x.as<double>(), center.rl, center.ql, next.rr, next.qr, opts.chi_max, true, N, C);
    // Extension One: every further eigenvector of the last micro-step gives an update of
    // its own, sharing cores s..b-1 with this one
    for (size_t q = 0; q < more.size(); ++q) {
      Sub A;
      A.s = S.s;
      A.t = S.t;
      for (const Core& m0 : S.mod) {
        Core cp;
        cp.rl = m0.rl; cp.rr = m0.rr; cp.ql = m0.ql; cp.qr = m0.qr;
        cp.d.ensure(m0.d.n);
        HC(hipMemcpyAsync(cp.d.p, m0.d.p, m0.d.n, hipMemcpyDeviceToDevice, stream));
        A.mod.push_back(std::move(cp));
      }
      Core Nq, Cq;
      split_two_site(*this, more[q].as<double>(), center.rl, center.ql, next.rr, next.qr, opts.chi_max, true, Nq, Cq);
      const double nc = norm_dev(*this, Cq.d.as<double>(), Cq.elems());
      scale(Cq.d.as<double>(), 1.0 / nc, Cq.elems(), stream);
      A.mod.push_back(std::move(Nq));
      A.mod.push_back(std::move(Cq));
      S.alt.push_back(std::move(A));
    }
    ph[4] += now() - tph;
    if (b < blast) {
      tph = now();
      Env nl;
      env_left(*Lcur, N, N, b, nl);
      Lrun = std::move(nl);
      Lcur = &Lrun;
      if (lin) {
        Env nf;
        ov_left(*FLcur, N, src.Fc[b], nf);
        FLrun = std::move(nf);
        FLcur = &FLrun;
      }
      ph[5] += now() - tph;
    } else {
      double nc = norm_dev(*this, C.d.as<double>(), C.elems());
      scale(C.d.as<double>(), 1.0 / nc, C.elems(), stream);
    }
    S.mod.push_back(std::move(N));
    center = std::move(C);
  }
  S.mod.push_back(std::move(center));
  HC(hipStreamSynchronize(stream));
  if (verbose)
    std::fprintf(stderr,
                 "[tt] subdomain %d sites %d..%d: E=%.10f matvecs=%d | products %.2fs, set-up %.2fs, Davidson "
                 "%.2fs, splits %.2fs, env %.2fs\n",
                 j, s, e, S.E, S.matvecs, sec_heff, ph[2], ph[3], ph[4], ph[5]);
}

// One-site subdomain sweep (Algorithm 2, one-site branch, with the subdomains of
// Extension Two): starting from the s-orthogonal copy of the iterate, the micro-step at
// site k replaces the centre core by the lowest eigenvector of its one-site problem; for
// k < e a charge-block QR of it gives the left-orthogonal core N_k and moves the
// centre into site k + 1 (R V_{k+1}).  The update is (U.., N_s..N_{e-1}, C_e, V..), C_e
// of unit norm; bond dimensions are those of the iterate.
void Engine::solve_subdomain1(const Engine& src, int j, int s, int e, Sub& S) {
  double tph = 0.0;
  S = Sub();
  S.s = s;
  S.t = e;
  auto copy_core = [&](const Core& a, Core& b) {
    b.rl = a.rl; b.rr = a.rr; b.ql = a.ql; b.qr = a.qr;
    b.d.ensure(a.d.n);
    HC(hipMemcpyAsync(b.d.p, a.d.p, a.d.n, hipMemcpyDeviceToDevice, stream));
  };
  Core center;
  copy_core(src.Wc[s], center);
  Env Lrun;
  const Env* Lcur = &src.Lenv[s];
  const bool lin = opts.functional == 1;
  Env FLrun;
  const Env* FLcur = lin ? &src.FL[s] : nullptr;
  if (lin) scale(center.d.as<double>(), src.xscale, center.elems(), stream);
  for (int k = s; k <= e; ++k) {
    std::vector<DevMem> more;
    Davidson r = lin ? local_lin(*this, *Lcur, k, src.Renv[k + 1], center.d, center, nullptr, *FLcur, src.FR[k + 1],
                                 src.Fc[k], nullptr)
                     : local_eig1(*this, *Lcur, k, src.Renv[k + 1], center.d, center,
                                  k == e && opts.coarse_k > 1 ? &more : nullptr);
    S.matvecs += r.matvecs;
    S.matvecs64 += r.matvecs64;
    S.E = r.theta;
    S.converged = S.converged && r.converged;
    if (k < e) {
      tph = now();
      Core next;
      copy_core(src.Vc[k + 1], next);
      qr_left(*this, center, next);
      ph[4] += now() - tph;
      tph = now();
      Env nl;
      env_left(*Lcur, center, center, k, nl);
      Lrun = std::move(nl);
      Lcur = &Lrun;
      if (lin) {
        Env nf;
        ov_left(*FLcur, center, src.Fc[k], nf);
        FLrun = std::move(nf);
        FLcur = &FLrun;
      }
      ph[5] += now() - tph;
      S.mod.push_back(std::move(center));
      center = std::move(next);
    } else {
      if (lin) {
        // the coarse step only needs the direction of each update
        const double nc = norm_dev(*this, center.d.as<double>(), center.elems());
        if (nc > 0.0) scale(center.d.as<double>(), 1.0 / nc, center.elems(), stream);
      }
      // Extension One: every further eigenvector of the last micro-step gives an update
      // of its own, sharing cores s..e-1 with this one
      for (size_t q = 0; q < more.size(); ++q) {
        Sub A;
        A.s = S.s;
        A.t = S.t;
        for (const Core& m0 : S.mod) {
          Core cp;
          copy_core(m0, cp);
          A.mod.push_back(std::move(cp));
        }
        Core Cq;
        Cq.rl = center.rl; Cq.rr = center.rr; Cq.ql = center.ql; Cq.qr = center.qr;
        Cq.d = std::move(more[q]);
        A.mod.push_back(std::move(Cq));
        S.alt.push_back(std::move(A));
      }
      S.mod.push_back(std::move(center));
    }
  }
  HC(hipStreamSynchronize(stream));
  if (verbose)
    std::fprintf(stderr,
                 "[tt] one-site subdomain %d sites %d..%d: E=%.10f matvecs=%d | products %.2fs, set-up %.2fs, "
                 "Davidson %.2fs, QR %.2fs, env %.2fs\n",
                 j, s, e, S.E, S.matvecs, sec_heff, ph[2], ph[3], ph[4], ph[5]);
}

void Engine::absorb_counters(Engine& w) {
  for (int i = 0; i < NPH; ++i) {
    ph[i] += w.ph[i];
    w.ph[i] = 0.0;
  }
  flops_heff += w.flops_heff;
  sec_heff += w.sec_heff;
  w.flops_heff = w.sec_heff = 0.0;
  t_env_bs += w.t_env_bs;
  t_env_dense += w.t_env_dense;
  t_ov += w.t_ov;
  n_env_bs += w.n_env_bs;
  n_env_dense += w.n_env_dense;
  n_ov += w.n_ov;
  w.t_env_bs = w.t_env_dense = w.t_ov = 0.0;
  w.n_env_bs = w.n_env_dense = w.n_ov = 0;
  for (int k = 0; k < KT_SLOTS; ++k)
    for (int c = 0; c < 4; ++c) {
      kstat[k][c] += w.kstat[k][c];
      w.kstat[k][c] = 0.0;
    }
  warn = std::max(warn, w.warn);
  w.warn = 0;
}

void Engine::run_tasks(int ntask, const std::vector<double>& cost, const std::function<void(Engine&, int)>& fn) {
  int nw = opts.sub_workers > 0 ? opts.sub_workers : 4;
  if (oom_cap > 0) nw = std::min(nw, oom_cap);
  nw = std::max(1, std::min(nw, ntask));
  if (nw == 1) {
    for (int t = 0; t < ntask; ++t) fn(*this, t);
    HC(hipStreamSynchronize(stream));
    return;
  }
  // shared inputs were produced on this engine's stream
  HC(hipStreamSynchronize(stream));
  while ((int)workers.size() < nw) workers.emplace_back(new Engine(*this, (int)workers.size()));
  std::vector<int> order(ntask);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  for (int w = 0; w < nw; ++w) {
    Engine* W = workers[w].get();
    W->opts = opts;
    W->kt_on = kt_on;
    W->verbose = verbose;
    W->warn = 0;
  }
  std::atomic<int> next{0};
  std::vector<std::exception_ptr> errs(nw);
  // tasks a worker gave up on when the device ran out of memory: that worker frees its
  // workspaces and leaves, the others go on; the tasks are run again below
  std::mutex fmu;
  std::vector<int> failed;
  std::vector<char> oom(nw, 0);
  std::vector<std::thread> th;
  for (int w = 0; w < nw; ++w) {
    Engine* W = workers[w].get();
    th.emplace_back([&, W, w]() {
      try {
        HC(hipSetDevice(opts.device));
        tl_stream = W->stream;
        // blocks of a worker may outlive it (they move into the context's results), so
        // they record the context's allocator, which lives as long as they do
        set_thread_allocator(&ext, W->stream);
        for (;;) {
          const int i = next.fetch_add(1);
          if (i >= ntask) break;
          try {
            tl_alloc_budget = opts.worker_alloc_limit > 0 ? opts.worker_alloc_limit : -1;
            fn(*W, order[i]);
            tl_alloc_budget = -1;
          } catch (const DeviceOOM&) {
            tl_alloc_budget = -1;
            (void)hipStreamSynchronize(W->stream);
            {
              std::lock_guard<std::mutex> g(fmu);
              failed.push_back(order[i]);
            }
            oom[w] = 1;
            W->release_workspaces();
            break;
          }
        }
        HC(hipStreamSynchronize(W->stream));
      } catch (...) {
        tl_alloc_budget = -1;
        errs[w] = std::current_exception();
        next.store(ntask);  // the other workers stop after their current task
        (void)hipStreamSynchronize(W->stream);
      }
      tl_stream = nullptr;
      set_thread_allocator(nullptr, nullptr);
    });
  }
  for (auto& t : th) t.join();
  for (int w = 0; w < nw; ++w) absorb_counters(*workers[w]);
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
  // Every task is independent and writes only its own outputs, so a task that ran out of
  // memory, or was never started because all workers left, is run again from the start,
  // one after another on this engine once the workers have given their memory back.  The
  // arithmetic is the same, so is the result; later calls use as many workers as fitted.
  const int started = std::min(next.load(), ntask);
  for (int k = started; k < ntask; ++k) failed.push_back(order[k]);
  if (!failed.empty()) {
    int fitted = 0;
    for (int w = 0; w < nw; ++w) fitted += !oom[w];
    oom_cap = std::max(1, fitted);
    for (int w = 0; w < (int)workers.size(); ++w) workers[w]->release_workspaces();
    if (verbose)
      std::fprintf(stderr, "[tt] device memory ran out with %d concurrent tasks: %zu task(s) run again one after "
                   "another; later calls use at most %d workers\n", nw, failed.size(), oom_cap);
    std::sort(failed.begin(), failed.end());
    for (int j : failed) fn(*this, j);
    HC(hipStreamSynchronize(stream));
  }
}

void Engine::local_solve(int nsub, const int* lengths, double* Eloc, int* mv) {
  if (!have_mpo || !have_mps) throw std::logic_error("local_solve needs the MPO and the TT iterate");
  if (nsub <= 0 || nsub > TT_MAX_SUB) throw std::invalid_argument("bad number of subdomains");
  if ((long long)nsub * opts.coarse_k > TT_MAX_SUB)
    throw std::invalid_argument("nsub * coarse_k exceeds the coarse-space limit TT_MAX_SUB");
  int tot = 0;
  for (int j = 0; j < nsub; ++j) {
    if (lengths[j] <= 0) throw std::invalid_argument("subdomain lengths must be positive");
    tot += lengths[j];
  }
  if (tot != L) throw std::invalid_argument("subdomain lengths must sum to L");
  free_caches();
  double tph = now();
  // Step 1: LQ sweep; W[k] centres, V[k] right-orthogonal cores
  Vc.clear(); Vc.resize(L);
  Wc.clear(); Wc.resize(L);
  {
    Core cur;  // W_{L-1}
    cur.rl = U[L - 1].rl; cur.rr = U[L - 1].rr; cur.ql = U[L - 1].ql; cur.qr = U[L - 1].qr;
    cur.d.ensure(U[L - 1].d.n);
    HC(hipMemcpyAsync(cur.d.p, U[L - 1].d.p, U[L - 1].d.n, hipMemcpyDeviceToDevice, stream));
    auto copy_core = [&](const Core& a, Core& b) {
      b.rl = a.rl; b.rr = a.rr; b.ql = a.ql; b.qr = a.qr;
      b.d.ensure(a.d.n);
      HC(hipMemcpyAsync(b.d.p, a.d.p, a.d.n, hipMemcpyDeviceToDevice, stream));
    };
    copy_core(cur, Wc[L - 1]);
    for (int k = L - 1; k >= 1; --k) {
      Core prev;
      copy_core(U[k - 1], prev);
      Core w;
      copy_core(Wc[k], w);
      lq_right(*this, w, prev);
      Vc[k] = std::move(w);
      Wc[k - 1] = std::move(prev);
      if (Vc[k].rl != U[k - 1].rr) throw std::runtime_error("LQ sweep changed a bond dimension (rank-deficient iterate)");
    }
    HC(hipStreamSynchronize(stream));
  }
  ph[0] += now() - tph;
  tph = now();
  // environment caches: Lenv[k] at bond k from U (k = 0..L-1), Renv[k] from V (k = 2..L)
  Lenv.clear(); Lenv.resize(L + 1);
  Renv.clear(); Renv.resize(L + 1);
  {
    // keep left environments only where they are read: subdomain starts and bond L-1
    std::vector<char> need(L + 1, 0);
    int st = 0;
    for (int j = 0; j < nsub; ++j) {
      need[st] = 1;
      st += lengths[j];
    }
    need[L - 1] = 1;
    Env cur;
    env_unit(cur, 1);
    for (int k = 0; k + 1 < L; ++k) {
      if (need[k]) {
        Lenv[k].R = cur.R; Lenv[k].rb = cur.rb; Lenv[k].rk = cur.rk;
        Lenv[k].d.ensure(cur.d.n);
        HC(hipMemcpyAsync(Lenv[k].d.p, cur.d.p, cur.d.n, hipMemcpyDeviceToDevice, stream));
      }
      Env nx;
      env_left(cur, U[k], U[k], k, nx);
      cur = std::move(nx);
    }
    Lenv[L - 1] = std::move(cur);
    HC(hipStreamSynchronize(stream));
  }
  env_unit(Renv[L], 1);
  // a one-site problem at site k reads Renv[k + 1] (k >= 0), a two-site one at bond
  // (b, b + 1) Renv[b + 2]
  const int kmin = opts.one_site ? 1 : 2;
  for (int k = L - 1; k >= kmin; --k) env_right(Renv[k + 1], Vc[k], Vc[k], k, Renv[k]);
  if (opts.functional == 1) {
    // overlap environments with the right-hand side: FL at the subdomain starts (and the
    // whole chain <tau(U)|F>), FR at every bond the local problems read
    if (!have_rhs) throw std::logic_error("the linear-system functional needs tt_set_rhs");
    if (Fc.size() != (size_t)L || Fc[L - 1].qr != U[L - 1].qr)
      throw std::invalid_argument("right-hand side and iterate are in different sectors");
    FL.clear(); FL.resize(L + 1);
    FR.clear(); FR.resize(L + 1);
    std::vector<char> need(L + 1, 0);
    for (int j = 0, st = 0; j < nsub; ++j) {
      need[st] = 1;
      st += lengths[j];
    }
    Env cur;
    env_unit(cur, 1);
    for (int k = 0; k < L; ++k) {
      if (need[k]) {
        FL[k].R = cur.R; FL[k].rb = cur.rb; FL[k].rk = cur.rk;
        FL[k].d.ensure(cur.d.n);
        HC(hipMemcpyAsync(FL[k].d.p, cur.d.p, cur.d.n, hipMemcpyDeviceToDevice, stream));
      }
      Env nx;
      ov_left(cur, U[k], Fc[k], nx);
      cur = std::move(nx);
    }
    d2h(&uf, cur.d.p, sizeof(double), stream);
    env_unit(FR[L], 1);
    for (int k = L - 1; k >= 1; --k) ov_right(FR[k + 1], Vc[k], Fc[k], FR[k]);
    HC(hipStreamSynchronize(stream));
  }
  ph[1] += now() - tph;
  if (verbose)
    std::fprintf(stderr, "[tt] step 1 done: LQ sweep %.2fs, environments %.2fs\n", ph[0], ph[1]);
  // Step 2: the subdomain sweeps are independent of one another (they read the
  // Step-1 cores and environments only); with several workers each runs on a
  // worker engine of its own (a host thread and a HIP stream), longest first
  HC(hipStreamSynchronize(stream));
  subs.clear();
  subs.resize(nsub);
  std::vector<int> first(nsub);
  for (int j = 0, st = 0; j < nsub; ++j) {
    first[j] = st;
    st += lengths[j];
  }
  const double t2 = now();
  // work estimate: sum over the subdomain's bonds of r_left * r_right * (r_left + r_right)
  std::vector<double> cost(nsub, 0.0);
  for (int j = 0; j < nsub; ++j)
    for (int k = first[j]; k < first[j] + lengths[j] && k + 1 < L; ++k) {
      const double rl = U[k].rl, rr = U[k + 1].rr;
      cost[j] += rl * rr * (rl + rr);
    }
  run_tasks(nsub, cost, [&](Engine& W, int j) {
    if (opts.one_site) W.solve_subdomain1(*this, j, first[j], first[j] + lengths[j] - 1, subs[j]);
    else W.solve_subdomain(*this, j, first[j], first[j] + lengths[j] - 1, subs[j]);
  });
  ph[8] += now() - t2;
  for (int j = 0; j < nsub; ++j) {
    if (Eloc) Eloc[j] = subs[j].E;
    if (mv) mv[j] = subs[j].matvecs;
  }
  // coarse states in subdomain order, each subdomain's lowest update first
  std::vector<Sub> states;
  sub_base.assign(nsub, 0);
  for (int j = 0; j < nsub; ++j) {
    sub_base[j] = (int)states.size();
    std::vector<Sub> alt = std::move(subs[j].alt);
    subs[j].alt.clear();
    states.push_back(std::move(subs[j]));
    for (Sub& a : alt) states.push_back(std::move(a));
  }
  subs = std::move(states);
  have_local = true;
}

// ---------------------------------------------------------------------------
// Step 3 + Step 4
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Step 4's block TT of sum_j c_j U^j (state 0 the iterate, then the updates)
// ---------------------------------------------------------------------------
// Bond k (1..L-1) blocks: U (r_k), V (r_k, if some state ended before site k), and one
// block per state that straddles the bond (several when Extension One keeps more than
// one update of a subdomain).  Labels are those of the blocks in this order, so they
// are grouped by charge within each block only.
namespace {
struct BondLayout {
  int offU = -1, offV = -1, dim = 0;
  int rU = 0, rV = 0;
  std::vector<std::pair<int, int>> str;  // (state j, block offset)
  Labels q;
  int off_of(int j) const {
    for (const auto& p : str)
      if (p.first == j) return p.second;
    return -1;
  }
};
}  // namespace

void Engine::combination_tt(const std::vector<double>& c, std::vector<Core>& T) {
  const int P = (int)subs.size();
  std::vector<BondLayout> bl(L + 1);
  bl[0].dim = 1;
  bl[0].q = {Q2{0, 0}};
  bl[L].dim = 1;
  bl[L].q = {U[L - 1].qr[0]};
  for (int k = 1; k < L; ++k) {
    BondLayout& B = bl[k];
    int d = 0;
    B.offU = d; B.rU = U[k].rl; d += B.rU;
    B.q.insert(B.q.end(), U[k].ql.begin(), U[k].ql.end());
    bool anyV = false;
    for (int j = 1; j <= P; ++j)
      if (subs[j - 1].t <= k - 1) anyV = true;
    if (anyV) {
      B.offV = d; B.rV = Vc[k].rl; d += B.rV;
      B.q.insert(B.q.end(), Vc[k].ql.begin(), Vc[k].ql.end());
    }
    for (int j = 1; j <= P; ++j) {
      const Sub& Sj = subs[j - 1];
      if (Sj.s <= k - 1 && k <= Sj.t) {
        B.str.push_back({j, d});
        d += Sj.mod[k - Sj.s].rl;
        B.q.insert(B.q.end(), Sj.mod[k - Sj.s].ql.begin(), Sj.mod[k - Sj.s].ql.end());
      }
    }
    B.dim = d;
  }
  // A two-site subdomain that starts at the last site has no bond of its own and leaves
  // the iterate unchanged (its core is the iterate's), so its coefficient adds to c_0; a
  // one-site update of the last site is a state of its own.
  double c0 = c[0];
  if (!opts.one_site)
    for (int j = 1; j <= P; ++j)
      if (subs[j - 1].s == L - 1) c0 += c[j];
  T.clear();
  T.resize(L);
  for (int k = 0; k < L; ++k) {
    Core& C = T[k];
    C.rl = bl[k].dim; C.rr = bl[k + 1].dim; C.ql = bl[k].q; C.qr = bl[k + 1].q;
    C.d.resize_zero(sizeof(double) * C.elems(), stream);
    const int Crrp = C.rrp();
    auto put = [&](const Core& src, int row_off, int col_off, double alpha, bool acc = false) {
      // C[row_off + a][s][col_off + b] = alpha * src[a][s][b]  (acc: +=, where several
      // one-site updates of the same site close into the same block)
      double* dst = C.d.as<double>() + (long long)row_off * 4 * Crrp + col_off;
      copy3d(src.d.as<double>(), 4LL * src.rrp(), src.rrp(), dst, 4LL * Crrp, Crrp, src.rl, 4, src.rr, alpha, stream,
             acc);
    };
    const BondLayout& Bl = bl[k];
    const BondLayout& Br = bl[k + 1];
    if (k == 0) {
      put(U[0], 0, (k + 1 < L) ? Br.offU : 0, (k + 1 < L) ? 1.0 : c0);
      if (k + 1 < L)
        for (int j = 1; j <= P; ++j) {
          const Sub& Sj = subs[j - 1];
          if (Sj.s != 0) continue;
          if (Sj.t == 0) put(Sj.mod[0], 0, Br.offV >= 0 ? Br.offV : 0, c[j], true);
          else put(Sj.mod[0], 0, Br.off_of(j), 1.0);
        }
      continue;
    }
    if (k == L - 1) {
      put(U[L - 1], Bl.offU, 0, c0);
      if (Bl.offV >= 0) put(Vc[L - 1], Bl.offV, 0, 1.0);
      for (const auto& p : Bl.str) {
        const Sub& Sj = subs[p.first - 1];
        put(Sj.mod[k - Sj.s], p.second, 0, c[p.first]);
      }
      if (opts.one_site)
        for (int j = 1; j <= P; ++j)
          if (subs[j - 1].s == L - 1) put(subs[j - 1].mod[0], Bl.offU, 0, c[j], true);
      continue;
    }
    // interior site
    put(U[k], Bl.offU, Br.offU, 1.0);
    if (Bl.offV >= 0) put(Vc[k], Bl.offV, Br.offV, 1.0);
    for (const auto& p : Bl.str) {
      const Sub& Sj = subs[p.first - 1];
      const Core& mc = Sj.mod[k - Sj.s];
      if (k < Sj.t) put(mc, p.second, Br.off_of(p.first), 1.0);
      else put(mc, p.second, Br.offV, c[p.first]);  // k == t_j : close into the V chain
    }
    for (int j = 1; j <= P; ++j) {
      const Sub& Sj = subs[j - 1];
      if (Sj.s != k) continue;
      if (Sj.t > k) put(Sj.mod[0], Bl.offU, Br.off_of(j), 1.0);
      else put(Sj.mod[0], Bl.offU, Br.offV, c[j], true);  // a one-site update of site k alone
    }
  }
  HC(hipStreamSynchronize(stream));
}

void Engine::grouped_combination(const std::vector<double>& v, std::vector<Core>& W) {
  std::vector<Core> T;
  combination_tt(v, T);
  // stable permutation of every inner bond that groups its labels by charge
  std::vector<std::vector<int>> perm(L + 1);
  perm[0] = {0};
  perm[L] = {0};
  for (int k = 1; k < L; ++k) {
    const Labels& q = T[k].ql;
    perm[k].resize(q.size());
    std::iota(perm[k].begin(), perm[k].end(), 0);
    std::stable_sort(perm[k].begin(), perm[k].end(), [&](int a, int b) { return q[a] < q[b]; });
  }
  std::vector<DevMem> dperm(L + 1);
  for (int k = 0; k <= L; ++k) upload(dperm[k], perm[k].data(), perm[k].size() * sizeof(int), stream);
  W.clear();
  W.resize(L);
  for (int k = 0; k < L; ++k) {
    const Core& C = T[k];
    Core& D = W[k];
    D.rl = C.rl; D.rr = C.rr;
    D.ql.resize(C.rl);
    D.qr.resize(C.rr);
    for (int a = 0; a < C.rl; ++a) D.ql[a] = C.ql[perm[k][a]];
    for (int b = 0; b < C.rr; ++b) D.qr[b] = C.qr[perm[k + 1][b]];
    D.d.resize_zero(sizeof(double) * D.elems(), stream);
    permute_core(C.d.as<double>(), C.rrp(), dperm[k].as<int>(), dperm[k + 1].as<int>(), C.rl, C.rr, D.d.as<double>(),
                 D.rrp(), stream);
  }
  HC(hipStreamSynchronize(stream));
}

// z_i = <U^i|H|W(v)> for all coarse states i (eq. aux_mat-vec_prod with the structured
// combination W(v) = sum_j v_j U^j): one right-to-left chain <V_{>=k}|H|W_{>=k}> kept at
// the bonds where an update ends, one left-to-right chain <U_{<k}|H|W_{<k}> that every
// update branches off at its first site, through its own cores.
int Engine::coarse_apply(const std::vector<double>& v, std::vector<double>& z) {
  const int P = (int)subs.size();
  std::vector<Core> W;
  grouped_combination(v, W);
  int nupd = 0;
  auto copy_env = [&](const Env& a, Env& b) {
    b.R = a.R; b.rb = a.rb; b.rk = a.rk;
    b.d.ensure(a.d.n);
    HC(hipMemcpyAsync(b.d.p, a.d.p, a.d.n, hipMemcpyDeviceToDevice, stream));
  };
  std::vector<char> needR(L + 1, 0);
  for (const Sub& Sj : subs) needR[Sj.t + 1] = 1;
  std::map<int, Env> RW;
  {
    Env cur;
    env_unit(cur, 1);
    if (needR[L]) copy_env(cur, RW[L]);
    for (int k = L - 1; k >= 1; --k) {
      bool any = false;
      for (int q = 1; q <= k; ++q) any = any || needR[q];
      if (!any) break;
      Env nx;
      env_right(cur, Vc[k], W[k], k, nx);
      ++nupd;
      cur = std::move(nx);
      if (needR[k]) copy_env(cur, RW[k]);
    }
  }
  std::vector<int> order(P);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return subs[a].s < subs[b].s; });
  z.assign(P + 1, 0.0);
  Env lw;
  env_unit(lw, 1);
  int kpos = 0;
  for (int i : order) {
    const Sub& Si = subs[i];
    for (; kpos < Si.s; ++kpos) {
      Env nx;
      env_left(lw, U[kpos], W[kpos], kpos, nx);
      ++nupd;
      lw = std::move(nx);
    }
    Env e, tmp;
    const Env* cur = &lw;
    for (int k = Si.s; k <= Si.t; ++k) {
      env_left(*cur, Si.mod[k - Si.s], W[k], k, tmp);
      ++nupd;
      e = std::move(tmp);
      cur = &e;
    }
    z[i + 1] = env_close(e, RW.at(Si.t + 1));
  }
  for (; kpos < L; ++kpos) {
    Env nx;
    env_left(lw, U[kpos], W[kpos], kpos, nx);
    ++nupd;
    lw = std::move(nx);
  }
  d2h(&z[0], lw.d.p, sizeof(double), stream);
  return nupd;
}

static const Core& core_of(const Engine& E, int j, int k, bool V_suffix) {
  // Ũ^j (j >= 1): U_k for k < s_j, mod for s_j..t_j, V_k beyond
  const Engine::Sub& S = E.subs[j - 1];
  if (k < S.s) return E.U[k];
  if (k <= S.t) return S.mod[k - S.s];
  (void)V_suffix;
  return E.Vc[k];
}

int Engine::coarse_correct(double* Sout, double* Aout, double* cout, double* lam, double* Eout, int* rank,
                           double* disc) {
  if (!have_local) throw std::logic_error("coarse_correct needs a preceding local_solve");
  double tph = now();
  const int P = (int)subs.size();
  const int n = P + 1;
  const bool lin = opts.functional == 1;
  // Krylov coarse solve: the Hamiltonian matrix is not formed, only S (its products
  // with A go through coarse_apply)
  const bool kry = opts.coarse_krylov != 0;
  coarse_matvecs = 0;
  std::vector<double> S((size_t)n * n, 0.0), A((size_t)n * n, 0.0), bvec(n, 0.0);
  if (lin) bvec[0] = uf;
  // sum over the valid block of El[a][f] Er[a][f] (two one-channel environments at one bond)
  auto ov_close2 = [](Engine& W, const Env& El, const Env& Er) {
    if (El.rb != Er.rb || El.rk != Er.rk) throw std::runtime_error("overlap closure: shape mismatch");
    const int p = padr(El.rb), q = padr(El.rk);
    std::vector<double> a((size_t)p * q), b((size_t)p * q);
    download(a.data(), El.d, a.size() * sizeof(double), W.stream);
    download(b.data(), Er.d, b.size() * sizeof(double), W.stream);
    double t = 0.0;
    for (int i = 0; i < El.rb; ++i)
      for (int j = 0; j < El.rk; ++j) t += a[(size_t)i * q + j] * b[(size_t)i * q + j];
    return t;
  };
  // <U0|H|U0> and <U0|U0> = 1 (normalised iterate)
  if (!kry) {
    Env e;
    env_left(Lenv[L - 1], U[L - 1], U[L - 1], L - 1, e);
    double v;
    d2h(&v, e.d.p, sizeof(double), stream);
    A[0] = v;
  }
  S[0] = 1.0;
  auto overlap_start = [](Engine& W, int rb, int rk, Env& e) {
    // identity on the bra/ket bond (both left-orthonormal prefixes of U)
    e.R = 1; e.rb = rb; e.rk = rk;
    const int p = padr(rb), q = padr(rk);
    std::vector<double> h((size_t)p * q, 0.0);
    for (int i = 0; i < std::min(rb, rk); ++i) h[(size_t)i * q + i] = 1.0;
    upload(e.d, h.data(), h.size() * sizeof(double), W.stream);
  };
  // overlap chains use a one-channel identity "MPO" through the same kernels
  SiteOp ident;
  {
    std::vector<int> o{0}, i{0};
    std::vector<double> op{1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    build_siteop(ident, 1, o, i, op, stream);
  }
  // the same chain through the block-sparse update (one neutral channel)
  BsSiteUse ident_use;
  if (opts.qn_skip) bs_site_use(*this, ident_use, ident, {Q2{0, 0}}, {Q2{0, 0}}, +1);
  HC(hipStreamSynchronize(stream));
  auto ov_left = [&](Engine& W, const Env& in, const Core& bra, const Core& ket, Env& out) {
    ScopeTimer tm(W, W.t_ov, W.n_ov);
    Env o;
    o.R = 1; o.rb = bra.rr; o.rk = ket.rr;
    o.d.ensure(sizeof(double) * o.elems());
    if (opts.qn_skip && in.rb == bra.rl && in.rk == ket.rl &&
        bs_env(W, ident_use, in.d.as<double>(), bra, ket, o.d.as<double>())) {
      out = std::move(o);
      return;
    }
    W.env_left_raw(padr(in.rb), padr(in.rk), bra.rrp(), ket.rrp(), 1, in.d.as<double>(), bra.d.as<double>(),
                   ket.d.as<double>(), ident, 1, o.d.as<double>());
    out = std::move(o);
  };
  auto ov_close = [](Engine& W, const Env& e) {
    // trace over the bond (the V suffix is right-orthonormal)
    const int p = padr(e.rb), q = padr(e.rk);
    std::vector<double> h((size_t)p * q);
    download(h.data(), e.d, h.size() * sizeof(double), W.stream);
    double t = 0.0;
    for (int i = 0; i < std::min(e.rb, e.rk); ++i) t += h[(size_t)i * q + i];
    return t;
  };
  // entries (0, j) and (j, j) of subdomain j
  auto column0_and_diag = [&](Engine& W, int j) {
    const Sub& Sj = subs[j - 1];
    // bra U^0 in the s_j-orthogonal gauge: W_{s_j}, V_{s_j+1}, ...
    Env eH, eS, tH, tS;
    const Env* cH = &Lenv[Sj.s];
    overlap_start(W, Wc[Sj.s].rl, Sj.mod[0].rl, eS);
    for (int k = Sj.s; k <= Sj.t; ++k) {
      const Core& bra = (k == Sj.s) ? Wc[k] : Vc[k];
      const Core& ket = Sj.mod[k - Sj.s];
      if (!kry) {
        W.env_left(*cH, bra, ket, k, tH);
        eH = std::move(tH);
        cH = &eH;
      }
      ov_left(W, eS, bra, ket, tS);
      eS = std::move(tS);
    }
    if (!kry) A[j] = A[(size_t)j * n] = W.env_close(eH, Renv[Sj.t + 1]);
    S[j] = S[(size_t)j * n] = ov_close(W, eS);
    // diagonal
    cH = &Lenv[Sj.s];
    overlap_start(W, Sj.mod[0].rl, Sj.mod[0].rl, eS);
    for (int k = Sj.s; k <= Sj.t; ++k) {
      const Core& c = Sj.mod[k - Sj.s];
      if (!kry) {
        W.env_left(*cH, c, c, k, tH);
        eH = std::move(tH);
        cH = &eH;
      }
      ov_left(W, eS, c, c, tS);
      eS = std::move(tS);
    }
    if (!kry) A[(size_t)j * n + j] = W.env_close(eH, Renv[Sj.t + 1]);
    S[(size_t)j * n + j] = ov_close(W, eS);
    if (lin) {
      // b_j = <U^j|F>: the overlap chain with F through the update's sites
      Env ef, tf;
      const Env* cf = &FL[Sj.s];
      for (int k = Sj.s; k <= Sj.t; ++k) {
        W.ov_left(*cf, Sj.mod[k - Sj.s], Fc[k], tf);
        ef = std::move(tf);
        cf = &ef;
      }
      bvec[j] = ov_close2(W, ef, FR[Sj.t + 1]);
    }
  };
  // entries (i, j), j > i: one chain with bra Ũ^i and ket U from bond s_i,
  // branching into ket Ũ^j at every later subdomain
  auto row = [&](Engine& W, int i) {
    const Sub& Si = subs[i - 1];
    Env cH, cS, tH, tS;
    bool first = true;
    int k = Si.s;
    for (int j = i + 1; j <= P; ++j) {
      const Sub& Sj = subs[j - 1];
      // advance the common chain to bond s_j
      for (; k < Sj.s; ++k) {
        const Core& bra = core_of(*this, i, k, true);
        const Core& ket = U[k];
        if (first) {
          if (!kry) W.env_left(Lenv[Si.s], bra, ket, k, tH);
          Env s0;
          overlap_start(W, bra.rl, ket.rl, s0);
          ov_left(W, s0, bra, ket, tS);
          first = false;
        } else {
          if (!kry) W.env_left(cH, bra, ket, k, tH);
          ov_left(W, cS, bra, ket, tS);
        }
        if (!kry) cH = std::move(tH);
        cS = std::move(tS);
      }
      // branch: sites s_j..t_j with ket = Ũ^j
      Env bH, bS, s0;
      const Env* pH = &cH;
      const Env* pS = &cS;
      if (first) {
        // Ũ^j starts at the same site as Ũ^i (an alternative update of the same
        // subdomain): the branch starts from the cached environment there
        pH = &Lenv[Si.s];
        overlap_start(W, core_of(*this, i, Sj.s, true).rl, Sj.mod[0].rl, s0);
        pS = &s0;
      }
      for (int kk = Sj.s; kk <= Sj.t; ++kk) {
        const Core& bra = core_of(*this, i, kk, true);
        const Core& ket = Sj.mod[kk - Sj.s];
        if (!kry) {
          W.env_left(*pH, bra, ket, kk, tH);
          bH = std::move(tH);
          pH = &bH;
        }
        ov_left(W, *pS, bra, ket, tS);
        bS = std::move(tS);
        pS = &bS;
      }
      if (!kry) A[(size_t)i * n + j] = A[(size_t)j * n + i] = W.env_close(bH, Renv[Sj.t + 1]);
      S[(size_t)i * n + j] = S[(size_t)j * n + i] = ov_close(W, bS);
    }
  };
  // tasks: P columns/diagonals, then P - 1 rows; cost = environment updates
  std::vector<double> cost;
  for (int j = 1; j <= P; ++j) cost.push_back(2.0 * (subs[j - 1].t - subs[j - 1].s + 1));
  for (int i = 1; i < P; ++i) {
    double c = 0.0;
    for (int j = i + 1; j <= P; ++j) c += subs[j - 1].t - subs[j - 1].s + 1;
    cost.push_back(2.0 * (c + std::max(0, subs[P - 1].s - subs[i - 1].s)));
  }
  run_tasks((int)cost.size(), cost, [&](Engine& W, int t) {
    if (t < P) column0_and_diag(W, t + 1);
    else row(W, t - P + 1);
  });
  ph[6] += now() - tph;
  tph = now();
  if (verbose) {
    const auto ps = pool().stats();
    const auto as = arena().stats();
    std::fprintf(stderr,
                 "[tt] step 3: coarse matrices %.2fs (so far: %d block-sparse env updates %.2fs, %d dense %.2fs, "
                 "%d overlap updates %.2fs; small blocks: %.0f allocations, %.1f GB, %.2fs; large-block chunks: "
                 "%.0f, %.1f GB, %.2fs)\n",
                 ph[6], n_env_bs, t_env_bs, n_env_dense, t_env_dense, n_ov, t_ov, ps[0], ps[1] / 1e9, ps[2], as[0],
                 as[1] / 1e9, as[2]);
  }
  // coarse eigenproblem (host FP64): canonical orthogonalisation of S
  std::vector<double> ws, Vs;
  jacobi_eig(n, S, ws, Vs);
  const double smax = ws[n - 1];
  std::vector<int> keep;
  for (int i = 0; i < n; ++i)
    if (ws[i] >= opts.coarse_eps * smax) keep.push_back(i);
  const int p = (int)keep.size();
  std::vector<double> X((size_t)n * p);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < p; ++a) X[(size_t)i * p + a] = Vs[(size_t)i * n + keep[a]] / std::sqrt(ws[keep[a]]);
  std::vector<double> c(n, 0.0);
  double lam_out = 0.0;
  std::vector<double> wa, Va;
  if (!kry) {
    std::vector<double> At((size_t)p * p, 0.0);
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b) {
        double v = 0.0;
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) v += X[(size_t)i * p + a] * A[(size_t)i * n + j] * X[(size_t)j * p + b];
        At[(size_t)a * p + b] = v;
      }
    for (int a = 0; a < p; ++a)
      for (int b = a + 1; b < p; ++b) {
        double v = 0.5 * (At[(size_t)a * p + b] + At[(size_t)b * p + a]);
        At[(size_t)a * p + b] = At[(size_t)b * p + a] = v;
      }
    jacobi_eig(p, At, wa, Va);
  }
  if (kry) {
    // Lanczos with full reorthogonalisation for the lowest eigenpair of X^T A X, started
    // from the iterate's coordinates in the orthonormal basis X (y_a = sum_i X_ia S_i0);
    // each product forms v = X y, z = A v through the combination TT, X^T z.  Stops when
    // the Ritz residual is <= 1e-12 max(1, |theta|) or the Krylov space is the whole space.
    auto red = [&](const std::vector<double>& y, std::vector<double>& out) {
      std::vector<double> v(n, 0.0), z;
      for (int i = 0; i < n; ++i)
        for (int a = 0; a < p; ++a) v[i] += X[(size_t)i * p + a] * y[a];
      coarse_apply(v, z);
      ++coarse_matvecs;
      out.assign(p, 0.0);
      for (int a = 0; a < p; ++a)
        for (int i = 0; i < n; ++i) out[a] += X[(size_t)i * p + a] * z[i];
    };
    std::vector<std::vector<double>> Q;
    std::vector<double> al, be;
    std::vector<double> q(p, 0.0);
    for (int a = 0; a < p; ++a)
      for (int i = 0; i < n; ++i) q[a] += X[(size_t)i * p + a] * S[(size_t)i * n];
    double nq = 0.0;
    for (double x : q) nq += x * x;
    nq = std::sqrt(nq);
    if (!(nq > 0.0)) {
      std::fill(q.begin(), q.end(), 0.0);
      q[0] = 1.0;
      nq = 1.0;
    }
    for (double& x : q) x /= nq;
    std::vector<double> ybest;
    double theta = 0.0;
    for (int m = 0; m < p; ++m) {
      Q.push_back(q);
      std::vector<double> w;
      red(q, w);
      double a_ = 0.0;
      for (int a = 0; a < p; ++a) a_ += q[a] * w[a];
      al.push_back(a_);
      for (int pass = 0; pass < 2; ++pass)
        for (const auto& qq : Q) {
          double d = 0.0;
          for (int a = 0; a < p; ++a) d += qq[a] * w[a];
          for (int a = 0; a < p; ++a) w[a] -= d * qq[a];
        }
      double b_ = 0.0;
      for (double x : w) b_ += x * x;
      b_ = std::sqrt(b_);
      // tridiagonal T_m and its lowest eigenpair
      const int mm = m + 1;
      std::vector<double> Tm((size_t)mm * mm, 0.0), wt, Vt;
      for (int r = 0; r < mm; ++r) {
        Tm[(size_t)r * mm + r] = al[r];
        if (r + 1 < mm) Tm[(size_t)r * mm + r + 1] = Tm[(size_t)(r + 1) * mm + r] = be[r];
      }
      jacobi_eig(mm, Tm, wt, Vt);
      theta = wt[0];
      ybest.assign(p, 0.0);
      for (int r = 0; r < mm; ++r)
        for (int a = 0; a < p; ++a) ybest[a] += Vt[(size_t)r * mm] * Q[r][a];
      const double res = b_ * std::fabs(Vt[(size_t)(mm - 1) * mm]);
      if (res <= 1e-12 * std::max(1.0, std::fabs(theta)) || b_ <= 1e-14 * std::max(1.0, std::fabs(theta))) break;
      be.push_back(b_);
      for (int a = 0; a < p; ++a) q[a] = w[a] / b_;
    }
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < p; ++a) c[i] += X[(size_t)i * p + a] * ybest[a];
    int imax = 0;
    for (int i = 1; i < n; ++i)
      if (std::fabs(c[i]) > std::fabs(c[imax])) imax = i;
    if (c[imax] < 0)
      for (double& v : c) v = -v;
    lam_out = theta;
    // the Hamiltonian matrix was not formed
    std::fill(A.begin(), A.end(), std::numeric_limits<double>::quiet_NaN());
  } else if (!lin) {
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < p; ++a) c[i] += X[(size_t)i * p + a] * Va[(size_t)a * p];
    int imax = 0;
    for (int i = 1; i < n; ++i)
      if (std::fabs(c[i]) > std::fabs(c[imax])) imax = i;
    if (c[imax] < 0)
      for (double& v : c) v = -v;
    lam_out = wa[0];
  } else {
    // coarse linear system (X^T A X) y = X^T b on the numerical range of S, c = X y;
    // the coarse minimum of J is 1/2 c.Ac - b.c
    if (!(wa[0] > 0.0)) throw std::runtime_error("linear-system functional: the coarse operator is not positive definite");
    std::vector<double> rb(p, 0.0), y(p, 0.0);
    for (int a = 0; a < p; ++a)
      for (int i = 0; i < n; ++i) rb[a] += X[(size_t)i * p + a] * bvec[i];
    for (int m = 0; m < p; ++m) {
      double proj = 0.0;
      for (int a = 0; a < p; ++a) proj += Va[(size_t)a * p + m] * rb[a];
      for (int a = 0; a < p; ++a) y[a] += Va[(size_t)a * p + m] * proj / wa[m];
    }
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < p; ++a) c[i] += X[(size_t)i * p + a] * y[a];
    double cAc = 0.0, bc = 0.0;
    for (int i = 0; i < n; ++i) {
      bc += bvec[i] * c[i];
      for (int j = 0; j < n; ++j) cAc += c[i] * A[(size_t)i * n + j] * c[j];
    }
    lam_out = 0.5 * cAc - bc;
  }
  coarse_b = bvec;
  int status = (p < n) ? TT_WRANKDEF : TT_OK;
  if (Sout) std::copy(S.begin(), S.end(), Sout);
  if (Aout) std::copy(A.begin(), A.end(), Aout);
  if (cout) std::copy(c.begin(), c.end(), cout);
  if (lam) *lam = lam_out;
  if (rank) *rank = p;

  // ---- Step 4: block TT of sum_j c_j Ũ^j and TT rounding ----
  std::vector<Core> T;
  combination_tt(c, T);
  HC(hipStreamSynchronize(stream));
  const double tc0 = now();
  // right-to-left orthogonalisation
  for (int k = L - 1; k >= 1; --k) lq_right(*this, T[k], T[k - 1]);
  const double tc1 = now();
  // left-to-right truncated SVD
  double discarded = 0.0;
  for (int k = 0; k + 1 < L; ++k) {
    Core& C = T[k];
    std::vector<int> rows, cols;
    Labels rq, cq;
    for (int a = 0; a < C.rl; ++a)
      for (int s = 0; s < 4; ++s) {
        rows.push_back(a * 4 + s);
        rq.push_back(qadd(C.ql[a], SITE_Q[s]));
      }
    for (int b = 0; b < C.rr; ++b) {
      cols.push_back(b);
      cq.push_back(C.qr[b]);
    }
    SectorSVD svd(*this);
    SvdOut o = svd.run(C.d.as<double>(), C.rrp(), rows, rq, cols, cq, opts.chi_max, true);
    discarded += o.discarded;
    const int kk = o.k, kp = padr(std::max(kk, 1));
    Core N;
    N.rl = C.rl; N.ql = C.ql; N.rr = kk; N.qr = o.q;
    N.d.resize_zero(sizeof(double) * (size_t)C.rlp() * 4 * kp, stream);
    DevMem SV;
    SV.resize_zero(sizeof(double) * (size_t)kp * C.rrp(), stream);
    svd.scatter(N.d.as<double>(), kp, SV.as<double>(), C.rrp(), 0);
    // next <- SV * next
    Core& Nx = T[k + 1];
    const int nrp = Nx.rrp();
    DevMem nd;
    nd.ensure(sizeof(double) * (size_t)kp * 4 * nrp);
    GemmArgs g{};
    g.M = kp; g.N = 4 * nrp; g.K = C.rrp(); g.batch = 1; g.kin = C.rrp();
    g.sAm = C.rrp(); g.sAkk = 1; g.sBkk = 4LL * nrp; g.sBn = 1; g.sCm = 4LL * nrp; g.alpha = 1.0; g.beta = 0.0;
    gemm<double>(g, SV.as<double>(), Nx.d.as<double>(), nd.as<double>(), true, true, stream);
    HC(hipStreamSynchronize(stream));
    Nx.d = std::move(nd);
    Nx.rl = kk;
    Nx.ql = o.q;
    T[k] = std::move(N);
  }
  double nr = norm_dev(*this, T[L - 1].d.as<double>(), T[L - 1].elems());
  if (!(nr > 0.0)) throw std::runtime_error("compressed iterate vanished");
  scale(T[L - 1].d.as<double>(), 1.0 / nr, T[L - 1].elems(), stream);
  HC(hipStreamSynchronize(stream));
  U = std::move(T);
  // the linear-system functional keeps the norm of the compressed combination
  if (lin) xscale = nr;
  free_caches();
  const double tc2 = now();
  double En = functional_value();
  ph[7] += now() - tph;
  if (verbose)
    std::fprintf(stderr,
                 "[tt] step 4: compressed in %.2fs (block TT %.2fs, LQ pass %.2fs, SVD pass %.2fs, energy %.2fs), "
                 "E=%.10f discarded=%.3g\n",
                 ph[7], tc0 - tph, tc1 - tc0, tc2 - tc1, now() - tc2, En, discarded);
  if (verbose) {
    std::fprintf(stderr, "[tt] batched SVDs of this context: %.3fs; bins (M x N: calls, matrices):", svd_seconds);
    for (auto& kv : svd_bins)
      std::fprintf(stderr, " %dx%d:%.0f,%.0f", kv.first.first, kv.first.second, kv.second[0], kv.second[1]);
    std::fprintf(stderr, "\n");
    svd_bins.clear();
    svd_seconds = 0.0;
  }
  if (Eout) *Eout = En;
  if (disc) *disc = discarded;
  return status;
}

// ---------------------------------------------------------------------------
// classical two-site DMRG (Algorithm 1)
// ---------------------------------------------------------------------------
void Engine::dmrg2(int nsweeps, double* energies) {
  if (!have_mpo || !have_mps) throw std::logic_error("dmrg2 needs the MPO and the TT iterate");
  // right-orthogonal start: cur = (W_0, V_1, ..., V_{L-1})
  std::vector<Core> cur(L);
  for (int k = 0; k < L; ++k) {
    cur[k].rl = U[k].rl; cur[k].rr = U[k].rr; cur[k].ql = U[k].ql; cur[k].qr = U[k].qr;
    cur[k].d.ensure(U[k].d.n);
    HC(hipMemcpyAsync(cur[k].d.p, U[k].d.p, U[k].d.n, hipMemcpyDeviceToDevice, stream));
  }
  for (int k = L - 1; k >= 1; --k) lq_right(*this, cur[k], cur[k - 1]);
  std::vector<Env> Le(L + 1), Re(L + 1);
  env_unit(Le[0], 1);
  env_unit(Re[L], 1);
  for (int k = L - 1; k >= 2; --k) env_right(Re[k + 1], cur[k], cur[k], k, Re[k]);
  DevMem x;
  int ie = 0;
  for (int sw = 0; sw < nsweeps; ++sw) {
    double th = 0.0;
    for (int b = 0; b + 1 < L; ++b) {
      two_site(*this, cur[b], cur[b + 1], x);
      Davidson r = local_eig(*this, Le[b], b, Re[b + 2], x, cur[b], cur[b + 1]);
      th = r.theta;
      Core N, C;
      split_two_site(*this, x.as<double>(), cur[b].rl, cur[b].ql, cur[b + 1].rr, cur[b + 1].qr, opts.chi_max, true,
                     N, C);
      cur[b] = std::move(N);
      cur[b + 1] = std::move(C);
      if (b + 2 < L) env_left(Le[b], cur[b], cur[b], b, Le[b + 1]);
    }
    if (energies) energies[ie++] = th;
    for (int b = L - 2; b >= 0; --b) {
      two_site(*this, cur[b], cur[b + 1], x);
      Davidson r = local_eig(*this, Le[b], b, Re[b + 2], x, cur[b], cur[b + 1]);
      th = r.theta;
      Core N, C;
      split_two_site(*this, x.as<double>(), cur[b].rl, cur[b].ql, cur[b + 1].rr, cur[b + 1].qr, opts.chi_max, false,
                     N, C);
      cur[b] = std::move(N);
      cur[b + 1] = std::move(C);
      if (b >= 1) env_right(Re[b + 2], cur[b + 1], cur[b + 1], b + 1, Re[b + 1]);
    }
    if (energies) energies[ie++] = th;
  }
  // back to left-orthogonal form
  for (int k = 0; k + 1 < L; ++k) qr_left(*this, cur[k], cur[k + 1]);
  double nr = norm_dev(*this, cur[L - 1].d.as<double>(), cur[L - 1].elems());
  scale(cur[L - 1].d.as<double>(), 1.0 / nr, cur[L - 1].elems(), stream);
  HC(hipStreamSynchronize(stream));
  U = std::move(cur);
  free_caches();
}

}  // namespace tt

// ---------------------------------------------------------------------------
// backward of E = <x|H_eff|x> (K12): the forward chain
//   T1 = L x, T2 = mix_W1(T1), T3 = mix_W2(T2), y = sum_C T3[C] R_C^T
// is linear in each operand, so every gradient is the contraction with that
// operand removed; the adjoint of a mix is the same gather with the entry
// lists regrouped by input channel and the local operators transposed.
// ---------------------------------------------------------------------------
namespace tt {

static std::vector<double> transpose_ops(const std::vector<double>& o) {
  std::vector<double> t(o.size());
  for (size_t e = 0; e < o.size() / 16; ++e)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) t[e * 16 + i * 4 + j] = o[e * 16 + j * 4 + i];
  return t;
}

void Engine::heff_grad_raw(int rl, int rr, int RA, int RB, int RC, const double* Lv, const double* Rv,
                           const std::vector<int>& A1, const std::vector<int>& B1, const std::vector<double>& o1,
                           const std::vector<int>& A2, const std::vector<int>& B2, const std::vector<double>& o2,
                           const double* x, double* En, double* gx, double* gL, double* gR, std::vector<double>& gop1,
                           std::vector<double>& gop2) {
  const long long slab = (long long)rl * 16 * rr;
  const size_t n = (size_t)slab;
  SiteOp w1f, w2f, w1fT, w2fT, w1a, w2a;
  std::vector<double> o1T = transpose_ops(o1), o2T = transpose_ops(o2);
  build_siteop(w1f, RB, B1, A1, o1, stream);
  build_siteop(w2f, RC, B2, A2, o2, stream);
  build_siteop(w1fT, RB, B1, A1, o1T, stream);
  build_siteop(w2fT, RC, B2, A2, o2T, stream);
  build_siteop(w1a, RA, A1, B1, o1T, stream);  // adjoint of mix 1: out A <- in B, op^T
  build_siteop(w2a, RB, A2, B2, o2T, stream);  // adjoint of mix 2: out B <- in C, op^T
  DevMem T1, T2, T3, G1, G2, G3, y, yT, LT, RT, ch1a, ch1b, ch2a, ch2b, g1d, g2d;
  T1.ensure(sizeof(double) * slab * RA);
  T2.ensure(sizeof(double) * slab * RB);
  T3.ensure(sizeof(double) * slab * RC);
  G3.ensure(sizeof(double) * slab * RC);
  G2.ensure(sizeof(double) * slab * RB);
  G1.ensure(sizeof(double) * slab * RA);
  y.ensure(sizeof(double) * n);
  yT.ensure(sizeof(double) * n);
  // forward
  GemmArgs g{};
  g.M = rl; g.N = 16 * rr; g.K = rl; g.batch = RA; g.kin = rl;
  g.sAb = (long long)rl * rl; g.sAm = rl; g.sAkk = 1; g.sBkk = 16LL * rr; g.sBn = 1;
  g.sCb = slab; g.sCm = 16LL * rr; g.alpha = 1.0; g.beta = 0.0;
  gemm<double>(g, Lv, x, T1.as<double>(), true, true, stream);
  mix<double>(RB, w1f.ptr.as<int>(), w1f.src.as<int>(), w1f.op64.as<double>(), T1.as<double>(), slab, T2.as<double>(),
              slab, rl, 4 * rr, stream);
  mix<double>(RC, w2f.ptr.as<int>(), w2f.src.as<int>(), w2f.op64.as<double>(), T2.as<double>(), slab, T3.as<double>(),
              slab, 4 * rl, rr, stream);
  GemmArgs h{};
  h.M = 16 * rl; h.N = rr; h.K = RC * rr; h.batch = 1; h.kin = rr;
  h.sAm = rr; h.sAkb = slab; h.sAkk = 1; h.sBkb = (long long)rr * rr; h.sBkk = 1; h.sBn = rr;
  h.sCm = rr; h.alpha = 1.0; h.beta = 0.0;
  gemm<double>(h, T3.as<double>(), Rv, y.as<double>(), true, false, stream);
  // E = x . y
  wsp.ensure(sizeof(double) * 264);
  DevMem part;
  part.ensure(sizeof(double) * kDotBlocks);
  multi_dot(x, n, 1, y.as<double>(), n, wsp.as<double>(), part.as<double>(), kDotBlocks, stream);
  d2h(En, wsp.p, sizeof(double), stream);
  // H^T x with every operand transposed
  LT.ensure(sizeof(double) * (size_t)RA * rl * rl);
  RT.ensure(sizeof(double) * (size_t)RC * rr * rr);
  transpose_batched(Lv, LT.as<double>(), RA, rl, rl, stream);
  transpose_batched(Rv, RT.as<double>(), RC, rr, rr, stream);
  heff<double>(rl, rr, RA, LT.as<double>(), w1fT, RB, w2fT, RC, RT.as<double>(), x, yT.as<double>(), nullptr, 0, 0);
  axpby(gx, 1.0, y.as<double>(), 1.0, yT.as<double>(), n, stream);
  // adjoint of the last GEMM: G3[C] = x R_C ; gR[C] = x^T T3[C]
  GemmArgs a{};
  a.M = 16 * rl; a.N = rr; a.K = rr; a.batch = RC; a.kin = rr;
  a.sAb = 0; a.sAm = rr; a.sAkk = 1; a.sBb = (long long)rr * rr; a.sBkk = rr; a.sBn = 1;
  a.sCb = slab; a.sCm = rr; a.alpha = 1.0; a.beta = 0.0;
  gemm<double>(a, x, Rv, G3.as<double>(), true, true, stream);
  GemmArgs b{};
  b.M = rr; b.N = rr; b.K = 16 * rl; b.batch = RC; b.kin = 16 * rl;
  b.sAb = 0; b.sAm = 1; b.sAkk = rr; b.sBb = slab; b.sBkk = rr; b.sBn = 1;
  b.sCb = (long long)rr * rr; b.sCm = rr; b.alpha = 1.0; b.beta = 0.0;
  gemm<double>(b, x, T3.as<double>(), gR, false, true, stream);
  // entry gradients of W2 and adjoint of mix 2
  const int nnz1 = (int)A1.size(), nnz2 = (int)A2.size();
  g2d.resize_zero(sizeof(double) * 16 * std::max(nnz2, 1), stream);
  g1d.resize_zero(sizeof(double) * 16 * std::max(nnz1, 1), stream);
  if (nnz2) {
    ch2a = upload_ints(B2, stream);  // G channel (output C)
    ch2b = upload_ints(A2, stream);  // T channel (input B)
    entry_grad<double>(nnz2, ch2a.as<int>(), ch2b.as<int>(), G3.as<double>(), slab, T2.as<double>(), slab, 4 * rl, rr,
                       g2d.as<double>(), stream);
  }
  mix<double>(RB, w2a.ptr.as<int>(), w2a.src.as<int>(), w2a.op64.as<double>(), G3.as<double>(), slab, G2.as<double>(),
              slab, 4 * rl, rr, stream);
  if (nnz1) {
    ch1a = upload_ints(B1, stream);
    ch1b = upload_ints(A1, stream);
    entry_grad<double>(nnz1, ch1a.as<int>(), ch1b.as<int>(), G2.as<double>(), slab, T1.as<double>(), slab, rl, 4 * rr,
                       g1d.as<double>(), stream);
  }
  mix<double>(RA, w1a.ptr.as<int>(), w1a.src.as<int>(), w1a.op64.as<double>(), G2.as<double>(), slab, G1.as<double>(),
              slab, rl, 4 * rr, stream);
  // gL[A] = G1[A] X^T
  GemmArgs c{};
  c.M = rl; c.N = rl; c.K = 16 * rr; c.batch = RA; c.kin = 16 * rr;
  c.sAb = slab; c.sAm = 16LL * rr; c.sAkk = 1; c.sBb = 0; c.sBkk = 1; c.sBn = 16LL * rr;
  c.sCb = (long long)rl * rl; c.sCm = rl; c.alpha = 1.0; c.beta = 0.0;
  gemm<double>(c, G1.as<double>(), x, gL, true, false, stream);
  HC(hipStreamSynchronize(stream));
  gop1.resize(16 * (size_t)nnz1);
  gop2.resize(16 * (size_t)nnz2);
  if (nnz1) d2h(gop1.data(), g1d.p, sizeof(double) * 16 * nnz1, stream);
  if (nnz2) d2h(gop2.data(), g2d.p, sizeof(double) * 16 * nnz2, stream);
}

// Gradient of E = <U|H|U> (normalised U fixed) with respect to every MPO entry:
//   dE/dW_k[A,s',s,B] = sum L_k[A][a'][a] U_k[a' s' b'] U_k[a s b] R_{k+1}[B][b'][b].
// Left environments are carried along the sweep; right environments are kept
// only at checkpoints every ~sqrt(L) sites and recomputed inside a segment.
void Engine::mpo_grad(double* En, double* const* gops) {
  if (!have_mpo || !have_mps) throw std::logic_error("gradient needs the MPO and the TT iterate");
  const int cstep = std::max(1, (int)std::ceil(std::sqrt((double)L)));
  std::map<int, Env> ckpt;  // right environments at checkpoint bonds
  {
    Env e;
    env_unit(e, 1);
    for (int k = L - 1; k >= 1; --k) {
      Env o;
      env_right(e, U[k], U[k], k, o);
      e = std::move(o);
      if (k % cstep == 0) {
        Env keep;
        keep.R = e.R; keep.rb = e.rb; keep.rk = e.rk;
        keep.d.ensure(e.d.n);
        HC(hipMemcpyAsync(keep.d.p, e.d.p, e.d.n, hipMemcpyDeviceToDevice, stream));
        ckpt[k] = std::move(keep);
      }
    }
  }
  std::map<int, Env> seg;  // right environments of the current segment
  auto right_env = [&](int bond) -> const Env& {
    if (bond == L) {
      if (!seg.count(L)) env_unit(seg[L], 1);
      return seg[L];
    }
    auto it = seg.find(bond);
    if (it != seg.end()) return it->second;
    auto ck = ckpt.find(bond);
    if (ck != ckpt.end()) return ck->second;
    // recompute from the next checkpoint at or above `bond`
    seg.clear();
    int top = L;
    for (auto& kv : ckpt)
      if (kv.first >= bond) { top = kv.first; break; }
    Env cur;
    if (top == L) env_unit(cur, 1);
    else {
      cur.R = ckpt[top].R; cur.rb = ckpt[top].rb; cur.rk = ckpt[top].rk;
      cur.d.ensure(ckpt[top].d.n);
      HC(hipMemcpyAsync(cur.d.p, ckpt[top].d.p, ckpt[top].d.n, hipMemcpyDeviceToDevice, stream));
    }
    for (int k = top - 1; k >= bond; --k) {
      Env o;
      env_right(cur, U[k], U[k], k, o);
      Env keep;
      keep.R = o.R; keep.rb = o.rb; keep.rk = o.rk;
      keep.d.ensure(o.d.n);
      HC(hipMemcpyAsync(keep.d.p, o.d.p, o.d.n, hipMemcpyDeviceToDevice, stream));
      seg[k] = std::move(keep);
      cur = std::move(o);
    }
    auto fin = seg.find(bond);
    if (fin == seg.end() || fin->second.d.p == nullptr) throw std::runtime_error("right environment missing");
    return fin->second;
  };
  Env Lk;
  env_unit(Lk, 1);
  for (int k = 0; k < L; ++k) {
    const SiteMPO& s = mpo[k];
    const Core& C = U[k];
    const Env& Rk = right_env(k + 1);
    const int rl = C.rlp(), rr = C.rrp();
    const long long sl = (long long)rl * 4 * rr;
    DevMem T, Rt, gd, cha, chb;
    T.ensure(sizeof(double) * sl * s.Rl);
    Rt.ensure(sizeof(double) * sl * s.Rr);
    GemmArgs g{};
    g.M = rl; g.N = 4 * rr; g.K = rl; g.batch = s.Rl; g.kin = rl;
    g.sAb = (long long)rl * rl; g.sAm = rl; g.sAkk = 1; g.sBkk = 4LL * rr; g.sBn = 1;
    g.sCb = sl; g.sCm = 4LL * rr; g.alpha = 1.0; g.beta = 0.0;
    gemm<double>(g, Lk.d.as<double>(), C.d.as<double>(), T.as<double>(), true, true, stream);
    GemmArgs h{};
    h.M = 4 * rl; h.N = rr; h.K = rr; h.batch = s.Rr; h.kin = rr;
    h.sAb = 0; h.sAm = rr; h.sAkk = 1; h.sBb = (long long)rr * rr; h.sBkk = rr; h.sBn = 1;
    h.sCb = sl; h.sCm = rr; h.alpha = 1.0; h.beta = 0.0;
    gemm<double>(h, C.d.as<double>(), Rk.d.as<double>(), Rt.as<double>(), true, true, stream);
    const int nnz = (int)s.A.size();
    gd.resize_zero(sizeof(double) * 16 * std::max(nnz, 1), stream);
    if (nnz) {
      cha = upload_ints(s.B, stream);
      chb = upload_ints(s.A, stream);
      entry_grad<double>(nnz, cha.as<int>(), chb.as<int>(), Rt.as<double>(), sl, T.as<double>(), sl, rl, rr,
                         gd.as<double>(), stream);
      d2h(gops[k], gd.p, sizeof(double) * 16 * nnz, stream);
    }
    Env o;
    env_left(Lk, C, C, k, o);
    Lk = std::move(o);
  }
  d2h(En, Lk.d.p, sizeof(double), stream);
}

// ---------------------------------------------------------------------------
// window operator with caller environments (the product used inside the local solves)
// ---------------------------------------------------------------------------
void Engine::window_apply(int b, int rl, int rr, const int32_t* ql, const int32_t* qr, const double* Lenv,
                          const double* Renv, int prec, const double* x, double* y) {
  if (!have_mpo) throw std::logic_error("window_apply needs the MPO");
  if (b < 0 || b + 1 >= L) throw std::invalid_argument("window site out of range");
  if (rl <= 0 || rr <= 0 || !ql || !qr || !Lenv || !Renv || !x || !y) throw std::invalid_argument("bad window operand");
  if (prec != TT_F64 && prec != TT_F32 && prec != TT_BF16) throw std::invalid_argument("bad precision");
  Labels lq(rl), rq(rr);
  for (int i = 0; i < rl; ++i) lq[i] = {ql[2 * i], ql[2 * i + 1]};
  for (int i = 0; i < rr; ++i) rq[i] = {qr[2 * i], qr[2 * i + 1]};
  Env Le, Re;
  Le.R = mpo[b].Rl; Le.rb = Le.rk = rl;
  Re.R = mpo[b + 1].Rr; Re.rb = Re.rk = rr;
  Le.d.borrow(const_cast<double*>(Lenv), sizeof(double) * Le.elems());
  Re.d.borrow(const_cast<double*>(Renv), sizeof(double) * Re.elems());
  Window w;
  prepare_window(*this, w, Le, b, Re, prec, lq, rq);
  window_matvec(*this, w, x, y, prec);
  HC(hipStreamSynchronize(stream));
}

}  // namespace tt
