// Orchestration of one subspace solve on the device, and the C ABI.
//
// Phase 1 (gates): every off-diagonal pair i < j gets its own copy of the
// left-canonical MPS j; the Givens network of U_i^T U_j is applied gate by
// gate, all pairs in lock step (the gate positions only depend on N).  A gate
// step is: exact LQ centre moves (if the run restarts further left), the
// two-site contraction with the gate, a per-quantum-number-block SVD, a host
// decision on the kept singular values (global top-chi per pair), and the
// split.  Phase 2 (environments): all pairs, including i = j, sweep bra x MPO
// x ket from left to right in a sector-padded common layout, so every pair
// shares one set of block descriptors.  Phase 3: the M x M eigenproblem.
#include "engine.hpp"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <functional>
#include <numeric>
#include <thread>
#include <sys/stat.h>
#include <unistd.h>
#include <tuple>

namespace tnqe {

// ------------------------------------------------------------ memory helpers
void *DevicePool::get(size_t bytes) {
  bytes = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
  if (arena_base_) {
    if (bytes > arena_size_ - arena_top_)
      throw Error(TNQE_EWORKSPACE, "workspace too small: " + std::to_string(arena_top_) + " bytes in use, " +
                                       std::to_string(bytes) + " more needed, " + std::to_string(arena_size_) +
                                       " available");
    void *p = arena_base_ + arena_top_;
    arena_starts_.push_back(arena_top_);
    order_.push_back(p);
    arena_top_ += bytes;
    arena_peak_ = std::max(arena_peak_, arena_top_);
    return p;
  }
  int best = -1;
  for (size_t i = 0; i < bufs_.size(); ++i)
    if (!bufs_[i].used && bufs_[i].n >= bytes && (best < 0 || bufs_[i].n < bufs_[best].n)) best = (int)i;
  if (best >= 0) {
    bufs_[best].used = true;
    order_.push_back(bufs_[best].p);
    return bufs_[best].p;
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    // free idle buffers and retry once
    for (size_t i = 0; i < bufs_.size();) {
      if (!bufs_[i].used) {
        (void)hipFree(bufs_[i].p);
        held_ -= bufs_[i].n;
        bufs_.erase(bufs_.begin() + i);
      } else {
        ++i;
      }
    }
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(TNQE_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
  }
  bufs_.push_back({p, bytes, true});
  order_.push_back(p);
  held_ += bytes;
  return p;
}

void DevicePool::rewind(size_t m) {
  if (arena_base_) {
    if (order_.size() > m) arena_top_ = arena_starts_[m];
    order_.resize(std::min(order_.size(), m));
    arena_starts_.resize(order_.size());
    return;
  }
  while (order_.size() > m) {
    void *p = order_.back();
    order_.pop_back();
    for (auto &b : bufs_)
      if (b.p == p) b.used = false;
  }
}

void DevicePool::release_all() {
  for (auto &b : bufs_) b.used = false;
  order_.clear();
  arena_starts_.clear();
  arena_top_ = 0;
}

void DevicePool::trim() {
  for (auto &b : bufs_) (void)hipFree(b.p);
  bufs_.clear();
  order_.clear();
  held_ = 0;
}

void DevicePool::set_arena(void *base, size_t bytes) {
  require(order_.empty(), TNQE_EINVAL, "device buffers still in use");
  char *b = static_cast<char *>(base);
  const size_t skip = (256 - reinterpret_cast<uintptr_t>(b) % 256) % 256;
  require(bytes >= skip, TNQE_EWORKSPACE, "workspace too small");
  arena_base_ = b + skip;
  arena_size_ = (bytes - skip) & ~size_t(255);
  arena_top_ = arena_peak_ = 0;
  arena_starts_.clear();
}

void DevicePool::clear_arena() {
  arena_base_ = nullptr;
  arena_size_ = arena_top_ = 0;
  arena_starts_.clear();
  order_.clear();
}

size_t DevicePool::available() const {
  return arena_base_ ? arena_size_ - arena_top_ : std::numeric_limits<size_t>::max();
}

// How long a waiting thread polls before it blocks: the per-ket loops of the
// gate phase come a fraction of a millisecond apart, and a wake-up through a
// condition variable costs tens of microseconds each time.
constexpr auto kPoolSpin = std::chrono::microseconds(200);

template <class Pred>
void spin_until(Pred done) {
  const auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; !done(); ++i)
    if ((i & 63) == 63 && std::chrono::steady_clock::now() - t0 > kPoolSpin) return;
}

ThreadPool::ThreadPool(int workers) {
  for (int i = 0; i < workers; ++i)
    threads_.emplace_back([this] {
      unsigned long long seen = 0;
      for (;;) {
        const std::function<void(int)> *f;
        int n;
        spin_until([&] { return stop_.load() || gen_.load() != seen; });
        {
          std::unique_lock<std::mutex> lk(m_);
          cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
          if (stop_) return;
          seen = gen_;
          // a job that has already returned (its caller cleared job_) is
          // skipped: its index counter may belong to the next job by now
          if (!job_) continue;
          f = job_;
          n = n_;
          ++busy_;
        }
        work(f, n);
        std::lock_guard<std::mutex> lk(m_);
        if (--busy_ == 0) done_cv_.notify_all();
      }
    });
}

ThreadPool::~ThreadPool() {
  {
    std::lock_guard<std::mutex> lk(m_);
    stop_ = true;
  }
  cv_.notify_all();
  for (auto &t : threads_) t.join();
}

void ThreadPool::work(const std::function<void(int)> *f, int n) {
  for (;;) {
    const int i = next_.fetch_add(1);
    if (i >= n) return;
    try {
      (*f)(i);
    } catch (...) {
      std::lock_guard<std::mutex> lk(m_);
      if (!err_) err_ = std::current_exception();
    }
  }
}

void ThreadPool::parallel_for(int n, const std::function<void(int)> &f) {
  if (n <= 0) return;
  if (threads_.empty() || n == 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  {
    std::lock_guard<std::mutex> lk(m_);
    job_ = &f;
    n_ = n;
    next_.store(0);
    err_ = nullptr;
    ++gen_;
  }
  cv_.notify_all();
  work(&f, n);
  spin_until([&] { return busy_.load() == 0 && next_.load() >= n; });
  std::unique_lock<std::mutex> lk(m_);
  done_cv_.wait(lk, [&] { return busy_ == 0 && next_.load() >= n_; });
  job_ = nullptr;
  if (err_) std::rethrow_exception(err_);
}

Staging::~Staging() {
  if (buf_) (void)hipHostFree(buf_);
  for (auto &o : old_) (void)hipHostFree(o.first);
}

void Staging::reset() {
  used_ = 0;
  for (auto &o : old_) (void)hipHostFree(o.first);
  old_.clear();
  heap_.clear();
}

void *Staging::put(const void *src, size_t bytes) {
  void *p = reserve(bytes);
  std::memcpy(p, src, bytes);
  return p;
}

void *Staging::reserve(size_t bytes) {
  const size_t need = (bytes + 255) & ~size_t(255);
  if (used_ + need > cap_) {
    if (!grow_) {
      // pageable host memory: kept until the next reset (copies may be in flight)
      heap_.emplace_back(new char[std::max<size_t>(need, 256)]);
      return heap_.back().get();
    }
    // keep the old buffer alive until the next reset (copies may be in flight)
    if (buf_) old_.push_back({buf_, cap_});
    cap_ = std::max<size_t>(need, std::max<size_t>(64u << 20, cap_ * 2));
    TNQE_HIP(hipHostMalloc((void **)&buf_, cap_, hipHostMallocDefault));
    used_ = 0;
  }
  char *p = buf_ + used_;
  used_ += need;
  return p;
}

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

ThreadPool &host_pool(tnqe_ctx *ctx);

struct Call {   // per-call helpers bound to a context
  tnqe_ctx *ctx;
  template <typename T>
  T *dev(size_t n) {
    return static_cast<T *>(ctx->pool.get(std::max<size_t>(1, n) * sizeof(T)));
  }
  template <typename T>
  T *upload(const std::vector<T> &v) {
    T *d = dev<T>(v.size());
    if (!v.empty()) {
      void *h = ctx->staging.put(v.data(), v.size() * sizeof(T));
      TNQE_HIP(hipMemcpyAsync(d, h, v.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
    }
    return d;
  }
  // several host arrays in one upload: add() returns each array's byte offset
  // (the arrays are copied once, straight into the pinned staging area, when
  // the blob is uploaded; they must live until then)
  struct Blob {
    struct Part {
      const void *src;
      size_t bytes, off;
    };
    std::vector<Part> parts;
    size_t size = 0;
    template <typename T>
    size_t add(const std::vector<T> &v) {
      const size_t off = (size + 255) & ~size_t(255);
      parts.push_back(Part{v.data(), v.size() * sizeof(T), off});
      size = off + std::max<size_t>(1, v.size()) * sizeof(T);
      return off;
    }
    template <typename T>
    size_t add(const std::vector<T> &&) = delete;   // the array must outlive the upload
  };
  char *upload(const Blob &b) {
    char *d = dev<char>(b.size);
    char *h = static_cast<char *>(ctx->staging.reserve(b.size));
    // large blobs are copied in 128 KiB pieces by the host workers
    constexpr size_t kPiece = 128 << 10;
    std::vector<std::pair<size_t, size_t>> pieces;   // (part, byte offset in the part)
    for (size_t i = 0; i < b.parts.size(); ++i)
      for (size_t o = 0; o < b.parts[i].bytes; o += kPiece) pieces.push_back({i, o});
    auto copy = [&](int k) {
      const Blob::Part &p = b.parts[pieces[k].first];
      const size_t o = pieces[k].second;
      std::memcpy(h + p.off + o, static_cast<const char *>(p.src) + o, std::min(kPiece, p.bytes - o));
    };
    if (pieces.size() > 2)
      host_pool(ctx).parallel_for((int)pieces.size(), copy);
    else
      for (size_t k = 0; k < pieces.size(); ++k) copy((int)k);
    TNQE_HIP(hipMemcpyAsync(d, h, b.size, hipMemcpyHostToDevice, ctx->stream));
    return d;
  }
  template <typename T>
  static T *at(char *base, size_t off) {
    return reinterpret_cast<T *>(base + off);
  }
  template <typename T>
  void upload_to(T *d, const T *src, size_t n) {
    if (n == 0) return;
    void *h = ctx->staging.put(src, n * sizeof(T));
    TNQE_HIP(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  }
  void sync() {
    TNQE_HIP(hipStreamSynchronize(ctx->stream));
    ctx->staging.reset();
  }
  void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(TNQE_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  }
};

// ------------------------------------------------------------ small host math
double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Givens plan: see the header of tnqe.h.  gates in application order.
void givens_plan(int N, const double *W, std::vector<int> &pos, std::vector<double> &theta, int &det_sign) {
  std::vector<double> Q(W, W + (size_t)N * N);
  std::vector<int> ea;
  std::vector<double> et;
  for (int c = 0; c + 1 < N; ++c)
    for (int r = N - 1; r > c; --r) {
      const int a = r - 1;
      const double x = Q[a * N + c], y = Q[r * N + c];
      // an entry that is zero to rounding is not rotated away (only the sign
      // of a negative pivot is fixed), so near-identity rotations plan as
      // near-identity networks instead of noise-driven angles
      double th;
      if (std::fabs(y) <= 1e-14)
        th = (a == c && x < 0.0) ? M_PI : 0.0;
      else
        th = std::atan2(-y, x);
      const double cs = std::cos(th), sn = std::sin(th);
      for (int col = 0; col < N; ++col) {
        const double qa = Q[a * N + col], qr = Q[r * N + col];
        Q[a * N + col] = cs * qa - sn * qr;
        Q[r * N + col] = sn * qa + cs * qr;
      }
      ea.push_back(a);
      et.push_back(th);
    }
  det_sign = (N == 0 || Q[(N - 1) * N + N - 1] > 0.0) ? 1 : -1;
  pos.assign(ea.rbegin(), ea.rend());
  theta.assign(et.rbegin(), et.rend());
}

// Spatial-orbital Givens gate on (k_p, k_{p+1}), built as the composite
// (1 x f2 x 1)(g2 x g2)(1 x f2 x 1) of App. A3 over the modes
// (p up, p dn, p+1 up, p+1 dn) and relabelled to k = n_up + 2 n_dn.
void gate_g4(double th, double out[256]) {
  const double c = std::cos(th), s = std::sin(th);
  for (int x = 0; x < 256; ++x) out[x] = gate4_entry(c, s, x);
}

// ------------------------------------------------------------ ket sets
// A batch of MPS being transformed on the device (one per off-diagonal pair,
// or one per input MPS during canonicalisation).
struct KetSet {
  Call *call = nullptr;
  int n = 0, N = 0, na = 0, nb = 0, nslot = 0;
  std::vector<int> cap;                 // capacity per bond
  std::vector<int> hdim;                // [bond][ket][slot]
  std::vector<int> htot;                // [bond][ket]
  std::vector<int2> hbtab;              // [bond][ket][slot]
  int2 *dbtab = nullptr;
  int *dbdim = nullptr;
  double *dsites = nullptr;
  std::vector<double *> site_ptr;       // [ket * N + p]
  double **dsite_ptr = nullptr;
  // one free site buffer per ket: a centre move writes the new left
  // neighbour there and frees the old one (all site buffers have the size of
  // the largest site)
  std::vector<double *> spare;
  std::vector<int64_t> site_cap;        // doubles per site

  int &dim(int b, int t, int s) { return hdim[((size_t)b * n + t) * nslot + s]; }
  int slot(int a, int bb) const { return (a < 0 || bb < 0 || a > na || bb > nb) ? -1 : a * (nb + 1) + bb; }
  int dim_q(int b, int t, int a, int bb) {
    const int s = slot(a, bb);
    return s < 0 ? 0 : dim(b, t, s);
  }
  int off_q(int b, int t, int a, int bb) {
    const int s = slot(a, bb);
    return s < 0 ? 0 : hbtab[((size_t)b * n + t) * nslot + s].x;
  }
  void init(Call *c, int nk, int N_, int na_, int nb_, const std::vector<int> &cap_) {
    call = c;
    n = nk;
    N = N_;
    na = na_;
    nb = nb_;
    nslot = (na + 1) * (nb + 1);
    cap = cap_;
    hdim.assign((size_t)(N + 1) * n * nslot, 0);
    htot.assign((size_t)(N + 1) * n, 0);
    hbtab.assign((size_t)(N + 1) * n * nslot, make_int2(0, 0));
    dbtab = call->dev<int2>(hbtab.size());
    dbdim = call->dev<int>(htot.size());
    site_cap.resize(N);
    int64_t stride = 0;
    for (int p = 0; p < N; ++p) {
      site_cap[p] = (int64_t)cap[p] * 4 * cap[p + 1];
      stride = std::max(stride, (site_cap[p] + 31) & ~int64_t(31));
    }
    dsites = call->dev<double>((size_t)stride * (N + 1) * n);
    site_ptr.resize((size_t)n * N);
    spare.resize(n);
    for (int t = 0; t < n; ++t) {
      for (int p = 0; p < N; ++p) site_ptr[(size_t)t * N + p] = dsites + ((size_t)t * (N + 1) + p) * stride;
      spare[t] = dsites + ((size_t)t * (N + 1) + N) * stride;
    }
    dsite_ptr = call->upload(site_ptr);
  }
  // offsets of the sectors of bond b from the current host dimensions,
  // [ket][slot] (prefix sums over the slots)
  std::vector<int> offsets(int b) {
    std::vector<int> o((size_t)n * nslot);
    for (int t = 0; t < n; ++t) {
      int acc = 0;
      for (int s = 0; s < nslot; ++s) {
        o[(size_t)t * nslot + s] = acc;
        acc += dim(b, t, s);
      }
    }
    return o;
  }
  // recompute offsets of bond b on the host and upload that slice (unless
  // the device table was already written by a kernel)
  void commit_bond(int b, bool upload = true) {
    for (int t = 0; t < n; ++t) {
      int o = 0;
      for (int s = 0; s < nslot; ++s) {
        const int d = dim(b, t, s);
        hbtab[((size_t)b * n + t) * nslot + s] = make_int2(o, d);
        o += d;
      }
      require(o <= cap[b], TNQE_ESHAPE, "bond dimension exceeds its capacity");
      htot[(size_t)b * n + t] = o;
    }
    if (!upload) return;
    call->upload_to(dbtab + (size_t)b * n * nslot, hbtab.data() + (size_t)b * n * nslot, (size_t)n * nslot);
    call->upload_to(dbdim + (size_t)b * n, htot.data() + (size_t)b * n, (size_t)n);
  }
  KetTables tables() const {
    KetTables k;
    k.site = dsite_ptr;
    k.btab = dbtab;
    k.bdim = dbdim;
    k.npair = n;
    k.N = N;
    k.na = na;
    k.nb = nb;
    k.nslot = nslot;
    return k;
  }
};

struct Scratch {
  int64_t used = 0;
  int64_t take(int64_t n) {
    const int64_t o = used;
    used += (n + 31) & ~int64_t(31);
    return o;
  }
};

// Work-unit prefix of a block list for the gate-phase kernels (first[0] = 0,
// first[n] = total units); units(b) gives a block's count.
template <class F>
std::vector<int> unit_prefix(const std::vector<Blk> &blks, F units) {
  std::vector<int> f(blks.size() + 1, 0);
  for (size_t i = 0; i < blks.size(); ++i) f[i + 1] = f[i] + units(blks[i]);
  return f;
}
Units units_at(char *base, size_t off, const std::vector<int> &f) {
  return Units{Call::at<const int>(base, off), (int)f.size() - 1, f.back()};
}

// Launch shape of the Jacobi SVD of an n-vector block with vectors of length
// m: ceil(n/2) processors of G lanes, E vector components per lane in
// registers (G E >= m), floor(n/2) traveller vectors in LDS rows of
// G (E + 2) doubles.
struct JacobiPlan {
  int kind = kJacobiGlobal, grp = 64, threads = 1024, mpad = 0;
  int64_t lds = 0;
};

JacobiPlan jacobi_plan(int n, int m) {
  JacobiPlan jp;
  const int P = (n + 1) / 2, NTr = n / 2;
  // preferred components per lane (tuning: TNQE_JACOBI_E = 4 ... 24; 8 was
  // the fastest at N = 24, chi = 256: more lanes per vector, shorter rounds)
  static const int target = [] {
    const char *e = std::getenv("TNQE_JACOBI_E");
    const int v = e ? std::atoi(e) : 8;
    return std::min(kJacobiMaxE, std::max(4, v / 4 * 4));
  }();
  int best = -1;
  for (int pass = 0; pass < 2 && best < 0; ++pass) {
    // first the smallest group with at most `target` components per lane,
    // else the smallest group that fits at all (fewest threads)
    const int cap = pass == 0 ? target : kJacobiMaxE;
    for (int G = 1; G <= 64; G *= 2) {
      const int E = ((m + G - 1) / G + 3) / 4 * 4;
      if (E > cap) continue;
      if (P * G > jacobi_max_threads(E)) break;
      const int64_t lds = ((int64_t)NTr * G * (E + 2) + NTr + n) * 8 + (int64_t)n * 4;
      if (lds > kJacobiLdsBytes) break;
      best = G;
      jp.kind = E / 4 - 1;
      jp.grp = G;
      jp.threads = (P * G + 63) / 64 * 64;
      jp.mpad = G * (E + 2);
      jp.lds = lds;
      break;
    }
  }
  // workgroups wider than `wide` threads take half the lanes per vector (twice
  // the components per lane, at most 16) when that fits: two such workgroups
  // then share a compute unit (tuning: TNQE_JACOBI_WIDE; at N = 24, chi = 256
  // 768 gave 1.36-1.38 s per solve, 512 1.39-1.40 s, no halving 1.43-1.44 s)
  static const int wide = [] {
    const char *e = std::getenv("TNQE_JACOBI_WIDE");
    return e ? std::atoi(e) : 768;
  }();
  if (best >= 2 && jp.threads > wide) {
    const int G = best / 2, E = ((m + G - 1) / G + 3) / 4 * 4;
    const int64_t lds = ((int64_t)NTr * G * (E + 2) + NTr + n) * 8 + (int64_t)n * 4;
    if (E <= 16 && P * G <= jacobi_max_threads(E) && lds <= kJacobiLdsBytes) {
      jp.kind = E / 4 - 1;
      jp.grp = G;
      jp.threads = (P * G + 63) / 64 * 64;
      jp.mpad = G * (E + 2);
      jp.lds = lds;
    }
  }
  return jp;
}

// plan the SVD of a block: launch shape and scratch (a global work area only
// for blocks the register/LDS kernels cannot hold)
// launch shape of a block (offW >= 0 marks the global-memory variant until
// its storage is assigned)
void plan_block(Blk &b) {
  b.n = std::min(b.R, b.C);
  require(b.n <= 1024, TNQE_ESHAPE, "quantum-number block larger than 1024 singular values");
  const JacobiPlan jp = jacobi_plan(b.n, std::max(b.R, b.C));
  b.grp = jp.grp;
  b.mpad = jp.mpad;
  b.offW = jp.kind == kJacobiGlobal ? 0 : -1;
}

// scratch of a planned block: T, U, B (and the work area of the global variant)
void take_block_storage(Blk &b, Scratch &sc) {
  const int m = std::max(b.R, b.C);
  b.offT = sc.take((int64_t)b.R * b.C);
  b.offU = sc.take((int64_t)b.R * b.n);
  b.offB = sc.take((int64_t)b.n * b.C);
  b.offS = -1;
  b.offW = b.offW >= 0 ? sc.take((int64_t)b.n * m + b.n) : -1;
}

// the launch shape plan_block chose, recovered from the block's group size
JacobiPlan planned_shape(const Blk &b) {
  JacobiPlan jp;
  if (b.offW >= 0) return jp;   // global-memory variant
  const int n = b.n, m = std::max(b.R, b.C), G = b.grp;
  const int E = ((m + G - 1) / G + 3) / 4 * 4, P = (n + 1) / 2, NTr = n / 2;
  jp.kind = E / 4 - 1;
  jp.grp = G;
  jp.threads = (P * G + 63) / 64 * 64;
  jp.mpad = b.mpad;
  jp.lds = ((int64_t)NTr * G * (E + 2) + NTr + n) * 8 + (int64_t)n * 4;
  return jp;
}


// Algorithmic flops of the SVD of an R x C block (n = min, m = max): the
// Gram-plus-symmetric-eigensolver count 2 n^2 m + 9 n^3 + 2 n^2 m.
double svd_flops(const Blk &b) {
  const double n = std::min(b.R, b.C), m = std::max(b.R, b.C);
  return 4.0 * n * n * m + 9.0 * n * n * n;
}

// TNQE_DEBUG_TIMING=1: host-side time split of the gate phase (diagnostics)
struct GateHostTiming {
  double sync_ms = 0.0, select_ms = 0.0, step_ms = 0.0, move_ms = 0.0;
  double build_ms = 0.0, two_site_ms = 0.0, svd_host_ms = 0.0, post_ms = 0.0;
  double plan_par_ms = 0.0, caller_ms = 0.0;
  int steps = 0;
};
double ms_between(std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}
GateHostTiming g_gate_timing;
bool debug_timing() {
  static const bool on = std::getenv("TNQE_DEBUG_TIMING") != nullptr;
  return on;
}

ThreadPool &host_pool(tnqe_ctx *ctx) {
  if (!ctx->pool_threads) {
    const int hw = (int)std::thread::hardware_concurrency();
    // tuning: TNQE_HOST_WORKERS sets the count of a context that has none
    static const int env = [] {
      const char *e = std::getenv("TNQE_HOST_WORKERS");
      return e ? std::max(0, std::min(63, std::atoi(e))) : -1;
    }();
    const int dflt = env >= 0 ? env : std::max(0, std::min(15, hw - 1));
    const int n = ctx->host_workers >= 0 ? ctx->host_workers : dflt;
    ctx->pool_threads = std::make_unique<ThreadPool>(n);
  }
  return *ctx->pool_threads;
}

// Device time of timed factorisation launches (per kernel, and per use:
// truncations or centre moves), collected after the next stream sync.
constexpr int kQrKind = kJacobiKinds;           // kind index of the Householder QR launches
constexpr int kFactKinds = kJacobiKinds + 1;
enum { kCatTrunc = 0, kCatMove = 1 };
struct SvdTimer {
  static constexpr int kMaxPending = 64;
  int npending = 0;
  int pending_kind[kMaxPending] = {}, pending_cat[kMaxPending] = {};
  double pending_flops[kMaxPending] = {};
  double ms = 0.0, flops = 0.0;
  int launches = 0;
  double kind_ms[kFactKinds] = {}, kind_flops[kFactKinds] = {};
  int kind_launches[kFactKinds] = {};
  double cat_ms[2] = {}, cat_flops[2] = {};
  int cat_launches[2] = {};
  // waits for the end events of the first `upto` pending launches, adds their
  // times, and moves the later ones (and their events) to the front
  void collect(tnqe_ctx *ctx, int upto = kMaxPending) {
    upto = std::min(upto, npending);
    for (int k = 0; k < upto; ++k) {
      float t = 0.0f;
      TNQE_HIP(hipEventSynchronize(ctx->svd_ev[2 * k + 1]));
      TNQE_HIP(hipEventElapsedTime(&t, ctx->svd_ev[2 * k], ctx->svd_ev[2 * k + 1]));
      ms += t;
      flops += pending_flops[k];
      ++launches;
      kind_ms[pending_kind[k]] += t;
      kind_flops[pending_kind[k]] += pending_flops[k];
      kind_launches[pending_kind[k]]++;
      cat_ms[pending_cat[k]] += t;
      cat_flops[pending_cat[k]] += pending_flops[k];
      cat_launches[pending_cat[k]]++;
    }
    for (int k = upto; k < npending; ++k) {
      std::swap(ctx->svd_ev[2 * (k - upto)], ctx->svd_ev[2 * k]);
      std::swap(ctx->svd_ev[2 * (k - upto) + 1], ctx->svd_ev[2 * k + 1]);
      pending_kind[k - upto] = pending_kind[k];
      pending_cat[k - upto] = pending_cat[k];
      pending_flops[k - upto] = pending_flops[k];
    }
    npending -= upto;
  }
  // a slot for the next launch, or -1 when all are pending (then untimed)
  int begin(tnqe_ctx *ctx, hipStream_t s, int kind, int cat, double fl) {
    if (npending >= kMaxPending) return -1;
    const int slot = npending;
    pending_flops[slot] = fl;
    pending_kind[slot] = kind;
    pending_cat[slot] = cat;
    TNQE_HIP(hipEventRecord(ctx->svd_ev[2 * slot], s));
    return slot;
  }
  void end(tnqe_ctx *ctx, hipStream_t s, int slot) {
    if (slot < 0) return;
    TNQE_HIP(hipEventRecord(ctx->svd_ev[2 * slot + 1], s));
    npending++;
  }
};

// Launch the SVDs of all blocks, grouped by kernel and workgroup size; within
// a launch the longest blocks go first.
void run_svd(Call &c, const Blk *dblk, const std::vector<Blk> &blks, int max_sweeps, double *scratch,
             SvdTimer *timer = nullptr, int cat = kCatTrunc, const std::vector<int> *subset = nullptr) {
  static const int kThreadSteps[6] = {64, 128, 256, 512, 768, 1024};
  std::map<std::pair<int, int>, std::vector<int>> groups;   // (kind, threads) -> blocks
  std::map<std::pair<int, int>, int64_t> lds;
  // TNQE_DEBUG_SVD=1: print the Jacobi sweep counts of every launch (diagnostics)
  static const bool dbg = std::getenv("TNQE_DEBUG_SVD") != nullptr;
  int *dsweeps = dbg ? c.dev<int>(blks.size()) : nullptr;
  std::vector<int64_t> work(blks.size()), sweep_cost(blks.size());
  const size_t nsel = subset ? subset->size() : blks.size();
  if (nsel == 0) return;
  for (size_t si = 0; si < nsel; ++si) {
    const size_t i = subset ? (size_t)(*subset)[si] : si;
    const Blk &b = blks[i];
    const int m = std::max(b.R, b.C);
    const JacobiPlan jp = planned_shape(b);
    int thr = 1024;
    for (int t : kThreadSteps)
      if (t >= jp.threads) {
        thr = t;
        break;
      }
    const auto key = std::make_pair(jp.kind, jp.kind == kJacobiGlobal ? 1024 : thr);
    groups[key].push_back((int)i);
    lds[key] = std::max(lds[key], jp.lds);
    work[i] = (int64_t)b.n * b.n * m;
    sweep_cost[i] = (int64_t)b.n * m;
  }
  // launches in decreasing estimated duration (longest processing time
  // first): the launch of the few largest blocks runs beside launches of many
  // small ones.  Duration estimate: the largest block's n m (rounds x vector
  // length) or the launch's total n^2 m spread over the chip, whichever is
  // larger.
  // Within a launch blocks go in decreasing n m (rounds per sweep times vector
  // length: the duration of a sweep at the launch's common lanes per vector;
  // measured 1.5-2 % faster per solve than decreasing n^2 m, n, or n m^2).
  std::vector<std::pair<double, std::pair<int, int>>> order;
  for (auto &kv : groups) {
    std::vector<int> &idx = kv.second;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return sweep_cost[x] > sweep_cost[y]; });
    double w = 0.0, lat = 0.0;
    for (int i : idx) {
      w += (double)work[i];
      lat = std::max(lat, (double)blks[i].n * std::max(blks[i].R, blks[i].C));
    }
    order.push_back({-std::max(lat, w / 2e4), kv.first});
  }
  std::sort(order.begin(), order.end());
  tnqe_ctx *ctx = c.ctx;
  if (timer && timer->npending + (int)order.size() > SvdTimer::kMaxPending) timer->collect(ctx);
  const int earlier = timer ? timer->npending : 0;
  const int nstream = std::min<int>(tnqe_ctx::kAux, (int)order.size());
  std::vector<const int *> didx(order.size());
  {
    Call::Blob bl;
    std::vector<size_t> off(order.size());
    for (size_t g = 0; g < order.size(); ++g) off[g] = bl.add(groups[order[g].second]);
    char *base = c.upload(bl);
    for (size_t g = 0; g < order.size(); ++g) didx[g] = Call::at<const int>(base, off[g]);
  }
  TNQE_HIP(hipEventRecord(ctx->fork_ev, ctx->stream));
  for (int i = 0; i < nstream; ++i) TNQE_HIP(hipStreamWaitEvent(ctx->aux[i], ctx->fork_ev, 0));
  // list scheduling: the first launches go to the side streams at once; each
  // further one (in the same order) is issued to whichever side stream has
  // finished its launch first, found by polling the event recorded after it.
  // Durations vary with the sweeps each block needs, so a launch assigned in
  // advance would often wait behind a long one while another stream is idle.
  auto issue = [&](size_t g, int si) {
    const auto key = order[g].second;
    const std::vector<int> &idx = groups[key];
    hipStream_t s = ctx->aux[si];
    int slot = -1;
    if (timer) {
      double f = 0.0;
      for (int i : idx) f += svd_flops(blks[i]);
      slot = timer->begin(ctx, s, key.first, cat, f);
    }
    launch_jacobi(dblk, didx[g], (int)idx.size(), key.first, key.second, (int)lds[key], scratch, max_sweeps,
                  dsweeps, s);
    if (timer) timer->end(ctx, s, slot);
    TNQE_HIP(hipEventRecord(ctx->join_ev[si], s));
  };
  size_t g = 0;
  for (int i = 0; i < nstream; ++i) issue(g++, i);
  while (g < order.size()) {
    for (int i = 0; i < nstream && g < order.size(); ++i) {
      const hipError_t q = hipEventQuery(ctx->join_ev[i]);
      if (q == hipSuccess) {
        issue(g++, i);
      } else if (q != hipErrorNotReady) {
        TNQE_HIP(q);
      }
    }
  }
  for (int i = 0; i < nstream; ++i) TNQE_HIP(hipStreamWaitEvent(ctx->stream, ctx->join_ev[i], 0));
  c.check_launch();
  // times of the earlier launches, while these run (the host would wait for
  // them anyway)
  if (timer) timer->collect(ctx, earlier);
  if (dbg) {
    std::vector<int> sw(blks.size());
    TNQE_HIP(hipMemcpyAsync(sw.data(), dsweeps, sw.size() * sizeof(int), hipMemcpyDeviceToHost, c.ctx->stream));
    TNQE_HIP(hipStreamSynchronize(c.ctx->stream));
    for (auto &kv : groups) {
      int mx = 0, at = kv.second[0];
      double mean = 0.0;
      for (int i : kv.second) {
        mean += sw[i];
        if (sw[i] > mx) { mx = sw[i]; at = i; }
      }
      std::fprintf(stderr, "svd kind %d threads %d: %zu blocks, sweeps mean %.1f max %d (block %dx%d)\n",
                   kv.first.first, kv.first.second, kv.second.size(), mean / kv.second.size(), mx, blks[at].R,
                   blks[at].C);
    }
  }
}

// Factorisations of the blocks of a centre move: Householder QR (one
// workgroup per block, in LDS) for every block that fits, the Jacobi SVD for
// the rest; blocks carry their choice in Blk::fact (set when planned).
void plan_move_block(Blk &b) {
  plan_block(b);
  b.fact = qr_lds_bytes(b) <= (size_t)kQrLdsBytes ? 1 : 0;
  if (b.fact) b.offW = -1;
}

double qr_flops(const Blk &b) {   // factorisation and formation of Q
  const double m = std::max(b.R, b.C), k = std::min(b.R, b.C);
  return 4.0 * m * k * k - 4.0 / 3.0 * k * k * k;
}

void factor_move(Call &c, const Blk *dblk, const std::vector<Blk> &blks, const int *dqr, const std::vector<int> &qr,
                 const std::vector<int> &svd, bool left, int max_sweeps, double *scratch, SvdTimer *timer) {
  tnqe_ctx *ctx = c.ctx;
  if (!qr.empty()) {
    size_t lds = 0;
    double fl = 0.0;
    for (int i : qr) {
      lds = std::max(lds, qr_lds_bytes(blks[i]));
      fl += qr_flops(blks[i]);
    }
    if (timer && timer->npending >= SvdTimer::kMaxPending) timer->collect(ctx);
    const int slot = timer ? timer->begin(ctx, ctx->stream, kQrKind, kCatMove, fl) : -1;
    launch_qr_blocks(dblk, dqr, (int)qr.size(), (int)lds, left, scratch, ctx->stream);
    if (timer) timer->end(ctx, ctx->stream, slot);
  }
  if (!svd.empty()) run_svd(c, dblk, blks, max_sweeps, scratch, timer, kCatMove, &svd);
}

struct TruncStats {
  std::vector<double> discarded;   // per ket, summed
  double min_gap = 1.0;
  int max_bond = 0;
  SvdTimer svd;                    // factorisations of the truncations and centre moves
  double move_wall_ms = 0.0;       // host time spent issuing centre moves in the gate phase
};

// One exact LQ centre move (site q -> q-1) for every ket in the set.
void move_left(KetSet &ks, int q, int max_sweeps, SvdTimer *timer) {
  Call &c = *ks.call;
  std::vector<std::vector<Blk>> pblk(ks.n);
  host_pool(c.ctx).parallel_for(ks.n, [&](int t) {
    for (int s = 0; s < ks.nslot; ++s) {
      const int d = ks.dim(q, t, s);
      if (d == 0) continue;
      const int sa = s / (ks.nb + 1), sb = s % (ks.nb + 1);
      Blk b{};
      b.pair = t;
      b.sa = sa;
      b.sb = sb;
      b.R = d;
      b.cs[0] = 0;
      for (int k = 0; k < 4; ++k) b.cs[k + 1] = b.cs[k] + ks.dim_q(q + 1, t, sa + qk_a(k), sb + qk_b(k));
      for (int k = 0; k <= 4; ++k) b.rs[k] = 0;
      b.C = b.cs[4];
      b.aux0 = ks.off_q(q, t, sa, sb);
      b.aux1 = ks.htot[(size_t)q * ks.n + t];
      if (b.C == 0) continue;
      plan_move_block(b);
      pblk[t].push_back(b);
    }
  });
  std::vector<Blk> blks;
  Scratch sc;
  for (int t = 0; t < ks.n; ++t)
    for (Blk &b : pblk[t]) {
      take_block_storage(b, sc);
      blks.push_back(b);
    }
  // new bond q: min(R, C) per sector
  for (int t = 0; t < ks.n; ++t)
    for (int s = 0; s < ks.nslot; ++s) ks.dim(q, t, s) = 0;
  for (Blk &b : blks) ks.dim(q, b.pair, ks.slot(b.sa, b.sb)) = b.n;
  for (Blk &b : blks) {
    b.offS = sc.take(b.n);
    b.kept = b.n;
  }
  {   // j0 in the new bond
    const std::vector<int> off = ks.offsets(q);
    for (Blk &b : blks) b.j0 = off[(size_t)b.pair * ks.nslot + ks.slot(b.sa, b.sb)];
  }
  double *scratch = c.dev<double>(sc.used);
  // the new left neighbour goes to each ket's spare site buffer and the old
  // one (read by the products, not copied) becomes the spare
  std::vector<double *> olds(ks.n);
  for (int t = 0; t < ks.n; ++t) {
    double *&cur = ks.site_ptr[(size_t)t * ks.N + q - 1];
    olds[t] = cur;
    cur = ks.spare[t];
    ks.spare[t] = olds[t];
  }
  const std::vector<int> u_gather =
      unit_prefix(blks, [](const Blk &b) { return gate_chunks((int64_t)b.R * b.C); });
  const std::vector<int> u_factor = unit_prefix(blks, [](const Blk &b) { return b.fact ? 0 : factor_units(b); });
  std::vector<int> qr, svd;
  for (size_t i = 0; i < blks.size(); ++i) (blks[i].fact ? qr : svd).push_back((int)i);
  // the new rows of A_q, then the tiles of the left neighbour's products
  // (bond q-1 is not changed by the move)
  const std::vector<int> u_apply = unit_prefix(blks, [&](const Blk &b) {
    int u = gate_chunks((int64_t)b.n * b.C);
    for (int k = 0; k < 4; ++k) u += gate_tiles(ks.dim_q(q - 1, b.pair, b.sa - qk_a(k), b.sb - qk_b(k)), b.n);
    return u;
  });
  Call::Blob bl;
  const size_t o_old = bl.add(olds), o_blk = bl.add(blks);
  const size_t o_ug = bl.add(u_gather), o_uf = bl.add(u_factor), o_ua = bl.add(u_apply);
  const size_t o_qr = bl.add(qr);
  char *base = c.upload(bl);
  double **d_old = Call::at<double *>(base, o_old);
  Blk *dblk = Call::at<Blk>(base, o_blk);
  const KetTables kt_old = ks.tables();
  launch_gather_lq(kt_old, q, dblk, units_at(base, o_ug, u_gather), scratch, c.ctx->stream);
  factor_move(c, dblk, blks, Call::at<const int>(base, o_qr), qr, svd, true, max_sweeps, scratch, timer);
  launch_svd_factor(dblk, units_at(base, o_uf, u_factor), scratch, c.ctx->stream);
  ks.commit_bond(q);
  // the site table with the swapped buffers, in stream order before the
  // kernel that writes the new neighbour
  c.upload_to(ks.dsite_ptr, ks.site_ptr.data(), ks.site_ptr.size());
  launch_apply_lq(ks.tables(), q, dblk, units_at(base, o_ua, u_apply), scratch, d_old, c.ctx->stream);
  c.check_launch();
}

// One exact QR centre move (site p -> p+1) for every ket in the set.
void move_right(KetSet &ks, int p, int max_sweeps, SvdTimer *timer) {
  Call &c = *ks.call;
  std::vector<Blk> blks;
  Scratch sc;
  for (int t = 0; t < ks.n; ++t) {
    for (int s = 0; s < ks.nslot; ++s) {
      const int d = ks.dim(p + 1, t, s);
      if (d == 0) continue;
      const int sa = s / (ks.nb + 1), sb = s % (ks.nb + 1);
      Blk b{};
      b.pair = t;
      b.sa = sa;
      b.sb = sb;
      b.C = d;
      b.rs[0] = 0;
      for (int k = 0; k < 4; ++k) b.rs[k + 1] = b.rs[k] + ks.dim_q(p, t, sa - qk_a(k), sb - qk_b(k));
      for (int k = 0; k <= 4; ++k) b.cs[k] = 0;
      b.R = b.rs[4];
      b.aux0 = ks.off_q(p + 1, t, sa, sb);
      b.aux1 = ks.htot[(size_t)(p + 1) * ks.n + t];
      if (b.R == 0) continue;
      plan_move_block(b);
      take_block_storage(b, sc);
      blks.push_back(b);
    }
  }
  for (int t = 0; t < ks.n; ++t)
    for (int s = 0; s < ks.nslot; ++s) ks.dim(p + 1, t, s) = 0;
  for (Blk &b : blks) ks.dim(p + 1, b.pair, ks.slot(b.sa, b.sb)) = b.n;
  for (Blk &b : blks) {
    b.offS = sc.take(b.n);
    b.kept = b.n;
  }
  {   // j0 in the new bond
    const std::vector<int> off = ks.offsets(p + 1);
    for (Blk &b : blks) b.j0 = off[(size_t)b.pair * ks.nslot + ks.slot(b.sa, b.sb)];
  }
  double *scratch = c.dev<double>(sc.used);
  std::vector<double *> olds(ks.n), srcs(ks.n);
  std::vector<int64_t> cnt(ks.n);
  double *oldbuf = c.dev<double>((size_t)ks.site_cap[p + 1] * ks.n);
  for (int t = 0; t < ks.n; ++t) {
    olds[t] = oldbuf + (size_t)t * ks.site_cap[p + 1];
    srcs[t] = ks.site_ptr[(size_t)t * ks.N + p + 1];
    cnt[t] = (int64_t)ks.htot[(size_t)(p + 1) * ks.n + t] * 4 * ks.htot[(size_t)(p + 2) * ks.n + t];
  }
  const std::vector<int> u_factor = unit_prefix(blks, [](const Blk &b) { return b.fact ? 0 : factor_units(b); });
  std::vector<int> qr, svd;
  for (size_t i = 0; i < blks.size(); ++i) (blks[i].fact ? qr : svd).push_back((int)i);
  Call::Blob bl;
  const size_t o_old = bl.add(olds), o_src = bl.add(srcs), o_cnt = bl.add(cnt), o_blk = bl.add(blks);
  const size_t o_uf = bl.add(u_factor), o_qr = bl.add(qr);
  char *base = c.upload(bl);
  double **d_old = Call::at<double *>(base, o_old);
  launch_copy(d_old, Call::at<double *>(base, o_src), Call::at<int64_t>(base, o_cnt), ks.n, c.ctx->stream);
  Blk *dblk = Call::at<Blk>(base, o_blk);
  launch_gather_qr(ks.tables(), p, dblk, (int)blks.size(), scratch, c.ctx->stream);
  factor_move(c, dblk, blks, Call::at<const int>(base, o_qr), qr, svd, false, max_sweeps, scratch, timer);
  launch_svd_factor(dblk, units_at(base, o_uf, u_factor), scratch, c.ctx->stream);
  ks.commit_bond(p + 1);
  launch_apply_qr(ks.tables(), p, dblk, (int)blks.size(), scratch, d_old, c.ctx->stream);
  c.check_launch();
}

// Gate at (a, a+1) for every ket with its own 16x16 matrix, then truncation.
void gate_step(KetSet &ks, int a, const std::vector<double> &gates, int chi_cap, double tau_w,
               int max_sweeps, bool renormalize, TruncStats &ts) {
  const auto tb0 = Clock::now();
  Call &c = *ks.call;
  // blocks of the new middle sectors (gated Theta) and of the old middle
  // sectors (two-site products) with their scratch, per ket on the host
  // workers (offsets relative to the ket's part of the scratch area)
  struct KetPlan {
    std::vector<Blk> blk, th;
    int64_t used = 0;
    int nv = 0;   // singular values of the ket
  };
  std::vector<KetPlan> kp(ks.n);
  host_pool(c.ctx).parallel_for(ks.n, [&](int t) {
    KetPlan &P = kp[t];
    Scratch sc;
    for (int s = 0; s < ks.nslot; ++s) {
      const int sa = s / (ks.nb + 1), sb = s % (ks.nb + 1);
      int rs[5] = {0, 0, 0, 0, 0};
      for (int k = 0; k < 4; ++k) rs[k + 1] = rs[k] + ks.dim_q(a, t, sa - qk_a(k), sb - qk_b(k));
      if (rs[4] == 0) continue;
      int cs[5] = {0, 0, 0, 0, 0};
      for (int k = 0; k < 4; ++k) cs[k + 1] = cs[k] + ks.dim_q(a + 2, t, sa + qk_a(k), sb + qk_b(k));
      if (cs[4] == 0) continue;
      Blk b{};
      b.pair = t;
      b.sa = sa;
      b.sb = sb;
      std::copy(rs, rs + 5, b.rs);
      std::copy(cs, cs + 5, b.cs);
      b.R = rs[4];
      b.C = cs[4];
      if (ks.dim_q(a + 1, t, sa, sb) > 0) {
        Blk bt = b;
        bt.offT = sc.take((int64_t)b.R * b.C);
        P.th.push_back(bt);
      }
      plan_block(b);
      take_block_storage(b, sc);
      b.offS = sc.take(b.n);
      P.nv += b.n;
      P.blk.push_back(b);
    }
    P.used = sc.used;
  });
  const auto tbp = Clock::now();
  // the kets' parts of the scratch area, block lists and first blocks
  std::vector<int64_t> kbase(ks.n + 1, 0);
  std::vector<int> kfirst(ks.n + 1, 0), tfirst(ks.n + 1, 0);
  int maxv = 0;
  for (int t = 0; t < ks.n; ++t) {
    kbase[t + 1] = kbase[t] + kp[t].used;
    kfirst[t + 1] = kfirst[t] + (int)kp[t].blk.size();
    tfirst[t + 1] = tfirst[t] + (int)kp[t].th.size();
    maxv = std::max(maxv, kp[t].nv);
  }
  std::vector<Blk> blks(kfirst[ks.n]), th(tfirst[ks.n]);
  std::vector<int> thidx((size_t)ks.n * ks.nslot, -1);
  host_pool(c.ctx).parallel_for(ks.n, [&](int t) {
    const int64_t o = kbase[t];
    for (size_t i = 0; i < kp[t].blk.size(); ++i) {
      Blk b = kp[t].blk[i];
      b.offT += o;
      b.offU += o;
      b.offB += o;
      b.offS += o;
      if (b.offW >= 0) b.offW += o;
      blks[kfirst[t] + i] = b;
    }
    for (size_t j = 0; j < kp[t].th.size(); ++j) {
      Blk b = kp[t].th[j];
      b.offT += o;
      th[tfirst[t] + j] = b;
      thidx[(size_t)t * ks.nslot + ks.slot(b.sa, b.sb)] = tfirst[t] + (int)j;
    }
  });
  Scratch sc;
  sc.used = kbase[ks.n];
  const auto tb1 = Clock::now();
  double *scratch = c.dev<double>(sc.used);
  const std::vector<int> u_gate =
      unit_prefix(blks, [](const Blk &b) { return gate_chunks((int64_t)b.R * b.C); });
  const std::vector<int> u_theta = unit_prefix(th, [](const Blk &b) { return gate_tiles(b.R, b.C); });
  // launch shapes of the factor and split kernels before the kept counts are
  // known (counted for all vectors)
  const std::vector<int> u_factor = unit_prefix(blks, factor_units);
  const std::vector<int> u_split = unit_prefix(blks, split_units);
  require(select_lds_bytes(maxv, ks.nslot) <= (size_t)kSelectLdsBytes, TNQE_ESHAPE,
          "too many singular values per ket for the truncation kernel");
  Call::Blob bl;
  const size_t o_g = bl.add(gates), o_b = bl.add(blks), o_t = bl.add(th), o_i = bl.add(thidx);
  const size_t o_ug = bl.add(u_gate), o_ut = bl.add(u_theta), o_uf = bl.add(u_factor), o_us = bl.add(u_split);
  const size_t o_kf = bl.add(kfirst);
  char *base = c.upload(bl);
  const double *dgates = Call::at<const double>(base, o_g);
  Blk *dblk = Call::at<Blk>(base, o_b);
  launch_two_site(ks.tables(), a, dblk, units_at(base, o_ug, u_gate), Call::at<const Blk>(base, o_t),
                  units_at(base, o_ut, u_theta), Call::at<const int>(base, o_i), dgates,
                  c.dev<double>((size_t)ks.n * 256), scratch,
                  c.ctx->stream);
  const auto tb2 = Clock::now();
  run_svd(c, dblk, blks, max_sweeps, scratch, &ts.svd);
  const auto tb3 = Clock::now();
  c.check_launch();
  // truncation on the device, then the factor and split kernels, queued
  // without a round trip through the host
  tnqe_ctx *ctx = c.ctx;
  const int nblk = (int)blks.size();
  // per-ket statistics and kept counts in one device buffer (one copy back)
  double *dstats = c.dev<double>((size_t)3 * ks.n + ((size_t)nblk + 1) / 2);
  int *dkept = reinterpret_cast<int *>(dstats + (size_t)3 * ks.n);
  const KetTables kt_new = ks.tables();
  double *dscale = renormalize ? c.dev<double>(ks.n) : nullptr;
  launch_select(dblk, Call::at<const int>(base, o_kf), ks.n, maxv, scratch, chi_cap, tau_w, kt_new, a + 1, dkept,
                dstats, dscale, ctx->stream);
  TNQE_HIP(hipEventRecord(ctx->sel_ev, ctx->stream));
  launch_svd_factor(dblk, units_at(base, o_uf, u_factor), scratch, ctx->stream);
  launch_split_gate(kt_new, a, dblk, units_at(base, o_us, u_split), scratch, dscale, ctx->stream);
  c.check_launch();
  // kept counts and per-ket statistics to pinned host memory on a side
  // stream (the main stream goes on with the factor and split); the host
  // polls for them, then mirrors the new bond for the next step's planning
  const size_t need = (size_t)3 * ks.n + ((size_t)nblk + 1) / 2;
  double *hbuf = ctx->sv_host;
  if (ctx->sv_cap < need) {
    if (ctx->no_alloc) {
      ctx->sv_pageable.resize(need);
      hbuf = ctx->sv_pageable.data();
    } else {
      if (ctx->sv_host) TNQE_HIP(hipHostFree(ctx->sv_host));
      ctx->sv_host = nullptr;
      ctx->sv_cap = 0;
      const size_t cap = std::max<size_t>(need * 2, 1 << 16);
      TNQE_HIP(hipHostMalloc((void **)&ctx->sv_host, cap * sizeof(double), hipHostMallocDefault));
      ctx->sv_cap = cap;
      hbuf = ctx->sv_host;
    }
  }
  double *hstats = hbuf;
  int *hkept = reinterpret_cast<int *>(hbuf + (size_t)3 * ks.n);
  TNQE_HIP(hipStreamWaitEvent(ctx->aux[0], ctx->sel_ev, 0));
  TNQE_HIP(hipMemcpyAsync(hstats, dstats, ((size_t)3 * ks.n + ((size_t)nblk + 1) / 2) * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->aux[0]));
  TNQE_HIP(hipEventRecord(ctx->sv_ev, ctx->aux[0]));
  const auto ts0 = Clock::now();
  for (;;) {
    const hipError_t q = hipEventQuery(ctx->sv_ev);
    if (q == hipSuccess) break;
    if (q != hipErrorNotReady) TNQE_HIP(q);
  }
  // every upload of this step has been consumed (the truncation ran after
  // all of them)
  ctx->staging.reset();
  const auto ts1 = Clock::now();
  for (int t = 0; t < ks.n; ++t)
    for (int s = 0; s < ks.nslot; ++s) ks.dim(a + 1, t, s) = 0;
  for (int i = 0; i < nblk; ++i) ks.dim(a + 1, blks[i].pair, ks.slot(blks[i].sa, blks[i].sb)) = hkept[i];
  ks.commit_bond(a + 1, false);
  for (int t = 0; t < ks.n; ++t) {
    ts.discarded[t] += hstats[3 * t + 1];
    ts.min_gap = std::min(ts.min_gap, hstats[3 * t + 2]);
    ts.max_bond = std::max(ts.max_bond, (int)hstats[3 * t]);
  }
  if (debug_timing()) {
    g_gate_timing.build_ms += ms_between(tb0, tb1);
    g_gate_timing.plan_par_ms += ms_between(tb0, tbp);
    g_gate_timing.two_site_ms += ms_between(tb1, tb2);
    g_gate_timing.svd_host_ms += ms_between(tb2, tb3);
    g_gate_timing.sync_ms += ms_between(ts0, ts1);
    g_gate_timing.select_ms += ms_between(ts1, Clock::now());
    g_gate_timing.steps++;
  }
}

// Device copy of the sparse groups' CSR structure for this MPO: cached in the
// context, or (calls that work in a caller's workspace) placed there.
const MpoDevice &mpo_dev_for(Call &c, const MpoStructure &mpo) {
  tnqe_ctx *ctx = c.ctx;
  if (!ctx->pool.arena()) {
    auto it = ctx->mpo_dev.find(mpo.N);
    if (it != ctx->mpo_dev.end()) return *it->second;
  }
  auto d = std::make_unique<MpoDevice>();
  std::vector<int> rp, cl;
  d->rp_off.resize(mpo.N);
  d->col_off.resize(mpo.N);
  for (int x = 0; x < mpo.N; ++x)
    for (const MpoGroup &g : mpo.groups[x]) {
      d->rp_off[x].push_back((int64_t)rp.size());
      d->col_off[x].push_back((int64_t)cl.size());
      rp.insert(rp.end(), g.rowptr.begin(), g.rowptr.end());
      cl.insert(cl.end(), g.col.begin(), g.col.end());
    }
  rp.push_back(0);
  cl.push_back(0);
  if (ctx->pool.arena()) {
    d->owned = false;
    d->rowptr = c.upload(rp);   // staged copies: the host vectors may go
    d->col = c.upload(cl);
    ctx->mpo_dev_call = std::move(d);
    return *ctx->mpo_dev_call;
  }
  TNQE_HIP(hipMalloc(&d->rowptr, rp.size() * sizeof(int)));
  TNQE_HIP(hipMalloc(&d->col, cl.size() * sizeof(int)));
  TNQE_HIP(hipMemcpy(d->rowptr, rp.data(), rp.size() * sizeof(int), hipMemcpyHostToDevice));
  TNQE_HIP(hipMemcpy(d->col, cl.data(), cl.size() * sizeof(int), hipMemcpyHostToDevice));
  const MpoDevice &ref = *d;
  ctx->mpo_dev[mpo.N] = std::move(d);
  return ref;
}

// ------------------------------------------------------------ environment sweep
// Tile shape for a list of problems with largest extents maxM x maxN.
// tile shapes of the environment GEMMs the autotuner times (tile modes 2 + k
// force candidate k on every GEMM list, for tests)
constexpr int kTileCands = 5;
constexpr int kTileCand[kTileCands][2] = {{256, 16}, {128, 32}, {64, 64}, {32, 128}, {16, 256}};

void pick_tile(int maxM, int maxN, bool long_m, int &tm, int &tn) {
  if (long_m) {
    if (maxN <= 16) { tm = 256; tn = 16; }
    else if (maxN <= 32) { tm = 128; tn = 32; }
    else { tm = 64; tn = 64; }
  } else {
    if (maxM <= 16) { tm = 16; tn = 256; }
    else if (maxM <= 32) { tm = 32; tn = 128; }
    else { tm = 64; tn = 64; }
  }
}

enum { kEnvG1 = 0, kEnvMix = 1, kEnvDense = 2, kEnvG2 = 3, kEnvFinal = 4, kEnvKinds = 5 };

struct EnvResult {
  std::vector<double> H, S;   // per env pair
  double flops = 0.0, bytes = 0.0, kernel_ms = 0.0, tune_ms = 0.0;
  double kind_ms[kEnvKinds] = {}, kind_flops[kEnvKinds] = {}, kind_bytes[kEnvKinds] = {};
  int kind_launches[kEnvKinds] = {};
  int max_pad = 0;
};

// Environment layout for given block-slot dimensions dpad[bond][slot]: the
// offset of every (class, ket sector) block of L at each bond, and per site
// the GEMM descriptors, channel-mix tasks and sources, dense couplings, tile
// shapes, X and Y sizes and the final-element terms.  Every size grows with
// dpad entry by entry, so the layout for an upper bound of the dimensions
// bounds the memory of the real one.  mdev may be null (sizes only).
struct EnvSiteTabs {
  std::vector<EnvG1> g1;
  std::vector<EnvG2> g2;
  int tm1 = 256, tn1 = 16, tm2 = 16, tn2 = 256;
  std::vector<std::vector<EnvGD>> dense;   // dense channel mixing, one level per launch
  std::vector<int> tmd, tnd;
  std::vector<MixTask> tasks;
  std::vector<MixSrc> srcs;
  std::vector<int> src_nnz;                // stored couplings of each source (work count)
  int64_t Xsize = 0, Ysize = 0;
  std::vector<EnvFinal> fin;
};

struct EnvLayout {
  std::vector<std::vector<int64_t>> Loff;  // [bond][class * nslot + slot], -1: none
  std::vector<int64_t> Lsize;              // [bond]
  std::vector<EnvSiteTabs> tabs;           // [site]
};

void plan_env_layout(const MpoStructure &mpo, const MpoDevice *mdev, int N, int na, int nb,
                     const std::vector<std::vector<int>> &dpad, ThreadPool &workers, EnvLayout &lay) {
  const int nslot = (na + 1) * (nb + 1), nb1 = nb + 1, nbond = N + 1;
  auto slot_of = [&](int a, int b) { return (a < 0 || b < 0 || a > na || b > nb) ? -1 : a * nb1 + b; };
  auto dp = [&](int b, int s) { return s < 0 ? 0 : dpad[b][s]; };
  std::vector<std::vector<int64_t>> &Loff = lay.Loff;
  std::vector<int64_t> &Lsize = lay.Lsize;
  Loff.assign(nbond, {});
  Lsize.assign(nbond, 0);
  const auto &cls = mpo.classes;
  for (int b = 0; b <= N; ++b) {
    Loff[b].assign(cls[b].size() * nslot, -1);
    int64_t o = 0;
    for (size_t ci = 0; ci < cls[b].size(); ++ci)
      for (int s = 0; s < nslot; ++s) {
        if (dpad[b][s] == 0) continue;
        const int sa = s / nb1, sb = s % nb1;
        const int sbra = slot_of(sa + cls[b][ci].da, sb + cls[b][ci].db);
        if (dp(b, sbra) == 0) continue;
        Loff[b][ci * nslot + s] = o;
        o += (int64_t)dpad[b][sbra] * cls[b][ci].nw * dpad[b][s];
      }
    Lsize[b] = o;
  }
  lay.tabs.assign(N, EnvSiteTabs{});
  std::vector<EnvSiteTabs> &tabs = lay.tabs;
  // sites are independent: their tables are built on the host workers
  workers.parallel_for(N, [&](int x) {
    EnvSiteTabs &tb = tabs[x];
    // GEMM1 and X slots
    std::vector<int64_t> offX(cls[x].size() * nslot * 4, -1);
    int64_t xo = 0;
    int maxM1 = 0, maxN1 = 0;
    for (size_t ci = 0; ci < cls[x].size(); ++ci)
      for (int s = 0; s < nslot; ++s) {
        const int64_t lo = Loff[x][ci * nslot + s];
        if (lo < 0) continue;
        const int sa = s / nb1, sb = s % nb1;
        const int sbra = slot_of(sa + cls[x][ci].da, sb + cls[x][ci].db);
        for (int k = 0; k < 4; ++k) {
          const int sk = slot_of(sa + qk_a(k), sb + qk_b(k));
          if (dp(x + 1, sk) == 0) continue;
          EnvG1 d{};
          d.x = x;
          d.nw = cls[x][ci].nw;
          d.sbra = sbra;
          d.s = s;
          d.k = k;
          d.sk = sk;
          d.offL = lo;
          d.offX = xo;
          offX[(ci * nslot + s) * 4 + k] = xo;
          const int Mp = dpad[x][sbra] * d.nw, Np = dpad[x + 1][sk];
          xo += ((int64_t)Mp * Np + 1) & ~(int64_t)1;   // even offsets: pairs of columns load as one vector
          maxM1 = std::max(maxM1, Mp);
          maxN1 = std::max(maxN1, Np);
          tb.g1.push_back(d);
        }
      }
    tb.Xsize = xo;
    pick_tile(maxM1, maxN1, true, tb.tm1, tb.tn1);
    // mix tasks and Y slots
    std::vector<int64_t> offY(cls[x + 1].size() * nslot * 4, -1);
    int64_t yo = 0;
    for (size_t co = 0; co < cls[x + 1].size(); ++co)
      for (int s = 0; s < nslot; ++s) {
        if (dpad[x + 1][s] == 0) continue;
        const int sa = s / nb1, sb = s % nb1;
        const int sbn = slot_of(sa + cls[x + 1][co].da, sb + cls[x + 1][co].db);
        if (dp(x + 1, sbn) == 0) continue;
        for (int kp = 0; kp < 4; ++kp) {
          const int s_a = slot_of(sa + cls[x + 1][co].da - qk_a(kp), sb + cls[x + 1][co].db - qk_b(kp));
          if (dp(x, s_a) == 0) continue;
          MixTask tk{};
          tk.x = x;
          tk.sa = s_a;
          tk.s = s;
          tk.nw_out = cls[x + 1][co].nw;
          tk.src0 = (int)tb.srcs.size();
          struct DenseSrc {
            int gi;
            int64_t offX;
            int nw_in;
            double f;
          };
          std::vector<DenseSrc> dsrc;
          for (size_t gi = 0; gi < mpo.groups[x].size(); ++gi) {
            const MpoGroup &g = mpo.groups[x][gi];
            if (g.cout != (int)co) continue;
            const OpPattern &P = mpo.patterns[g.pattern];
            for (int e = 0; e < P.n; ++e) {
              if (P.kp[e] != kp) continue;
              const int k = P.k[e];
              const int s_in = slot_of(sa - qk_a(k), sb - qk_b(k));
              if (s_in < 0) continue;
              const int64_t ox = offX[((size_t)g.cin * nslot + s_in) * 4 + k];
              if (ox < 0) continue;
              // the source block's bra sector must be the task's (shape of the read)
              const int s_src = slot_of(sa - qk_a(k) + cls[x][g.cin].da, sb - qk_b(k) + cls[x][g.cin].db);
              require(s_src == s_a, TNQE_EINVAL, "MPO transition breaks particle-number bookkeeping");
              if (g.dense) {
                dsrc.push_back({(int)gi, ox, cls[x][g.cin].nw, P.f[e]});
                continue;
              }
              MixSrc sr{};
              sr.offX = ox;
              sr.vbase = mpo.site_nnz_off[x] + g.val_off;
              sr.rp = mdev ? mdev->rp_off[x][gi] : 0;
              sr.cp = mdev ? mdev->col_off[x][gi] : 0;
              sr.nw_in = cls[x][g.cin].nw;
              sr.group = (int)gi;
              sr.factor = P.f[e];
              tb.srcs.push_back(sr);
              tb.src_nnz.push_back((int)g.col.size());
            }
          }
          tk.nsrc = (int)tb.srcs.size() - tk.src0;
          if (tk.nsrc == 0 && dsrc.empty()) continue;
          tk.offY = yo;
          offY[(co * nslot + s) * 4 + kp] = yo;
          const int64_t tot = (int64_t)dpad[x][s_a] * tk.nw_out * dpad[x + 1][s];
          yo += (tot + 1) & ~(int64_t)1;
          // dense sources accumulate after the sparse pass, one source of a
          // block per launch so no two problems of a launch share an output
          for (size_t q = 0; q < dsrc.size(); ++q) {
            const MpoGroup &g = mpo.groups[x][dsrc[q].gi];
            EnvGD d{};
            d.x = x;
            d.sa = s_a;
            d.s = s;
            d.nr = g.nr;
            d.nc = g.nc;
            d.r0 = g.r0;
            d.c0 = g.c0;
            d.nw_in = dsrc[q].nw_in;
            d.nw_out = tk.nw_out;
            d.offY = tk.offY;
            d.offX = dsrc[q].offX;
            d.valoff = mpo.site_nnz_off[x] + g.val_off;
            d.f = dsrc[q].f;
            if (tb.dense.size() <= q) tb.dense.resize(q + 1);
            tb.dense[q].push_back(d);
          }
          tb.tasks.push_back(tk);
        }
      }
    tb.Ysize = yo;
    for (auto &lv : tb.dense) {
      // N runs over (bra row, ket index) of the block
      int maxM = 0, maxN = 0;
      for (auto &d : lv) {
        maxM = std::max(maxM, d.nr);
        maxN = std::max(maxN, dpad[x][d.sa] * dpad[x + 1][d.s]);
      }
      int tm, tn;
      pick_tile(maxM, maxN, false, tm, tn);
      tb.tmd.push_back(tm);
      tb.tnd.push_back(tn);
    }
    if (x < N - 1) {
      int maxM2 = 0, maxN2 = 0;
      for (size_t co = 0; co < cls[x + 1].size(); ++co)
        for (int s = 0; s < nslot; ++s) {
          const int64_t lo = Loff[x + 1][co * nslot + s];
          if (lo < 0) continue;
          const int sa = s / nb1, sb = s % nb1;
          const int sbn = slot_of(sa + cls[x + 1][co].da, sb + cls[x + 1][co].db);
          EnvG2 d{};
          d.x = x;
          d.nw = cls[x + 1][co].nw;
          d.sbn = sbn;
          d.s = s;
          d.offL = lo;
          d.nseg = 0;
          for (int kp = 0; kp < 4; ++kp) {
            const int64_t oy = offY[(co * nslot + s) * 4 + kp];
            if (oy < 0) continue;
            d.sa[d.nseg] = slot_of(sa + cls[x + 1][co].da - qk_a(kp), sb + cls[x + 1][co].db - qk_b(kp));
            d.kp[d.nseg] = kp;
            d.offY[d.nseg] = oy;
            d.nseg++;
          }
          maxM2 = std::max(maxM2, dpad[x + 1][sbn]);
          maxN2 = std::max(maxN2, d.nw * dpad[x + 1][s]);
          tb.g2.push_back(d);
        }
      pick_tile(maxM2, maxN2, false, tb.tm2, tb.tn2);
    } else {
      const int sN = slot_of(na, nb);
      const int co = mpo.final_class;
      for (int kp = 0; kp < 4; ++kp) {
        const int64_t oy = offY[((size_t)co * nslot + sN) * 4 + kp];
        if (oy < 0) continue;
        EnvFinal f{};
        f.sa = slot_of(na - qk_a(kp), nb - qk_b(kp));
        f.kp = kp;
        f.offY = oy;
        tb.fin.push_back(f);
      }
    }
  });
}

// Environment sweeps of all pairs.  Items are the M bra MPS followed by the
// rotated kets; pair q contracts bra item pairs[q].first with its ket item.
// Block slots are sized by the largest dimensions over the items (one
// descriptor list for all pairs); the kernels use each pair's own extents.
// Tuned tile shapes: a text file of lines "kind bytes lgM lgN lgW tileM tileN"
// (TNQE_TUNE_FILE, else $HOME/.cache/tnqe_env_tiles.txt).
std::string tune_file() {
  if (const char *f = std::getenv("TNQE_TUNE_FILE")) return f;
  const char *h = std::getenv("HOME");
  return std::string(h ? h : ".") + "/.cache/tnqe_env_tiles.txt";
}

void load_tiles(tnqe_ctx *ctx) {
  if (ctx->tiles_loaded) return;
  ctx->tiles_loaded = true;
  FILE *f = std::fopen(tune_file().c_str(), "r");
  if (!f) return;
  int v[7];
  while (std::fscanf(f, "%d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6]) == 7)
    ctx->tiles[{v[0], v[1], v[2], v[3], v[4]}] = {v[5], v[6]};
  std::fclose(f);
}

void save_tiles(const tnqe_ctx *ctx) {
  const std::string path = tune_file(), tmp = path + ".tmp" + std::to_string((long)getpid());
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) return;   // the cache is an optimisation: an unwritable path is not an error
  for (const auto &kv : ctx->tiles)
    std::fprintf(f, "%d %d %d %d %d %d %d\n", kv.first[0], kv.first[1], kv.first[2], kv.first[3], kv.first[4],
                 kv.second.first, kv.second.second);
  std::fclose(f);
  if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

int ceil_log2(double v) {
  int l = 0;
  while ((double)(1ll << l) < v && l < 62) ++l;
  return l;
}

template <typename T>
void env_phase(Call &c, const tnqe_problem &pb, KetSet *kets, const std::vector<std::pair<int, int>> &pairs,
               const std::vector<int> &ket_of_pair, const MpoStructure &mpo, const double *dvals,
               int64_t nnz_total, EnvResult &res, int tile_mode = 0, int cm = 0) {
  hipStream_t st = c.ctx->stream;
  const auto tq0 = Clock::now();
  const int N = pb.N, M = pb.M, nslot = pb.nslot(), nbond = N + 1;
  const int nket = kets ? kets->n : 0;
  const int nitem = M + nket;
  // ---- item sector tables
  std::vector<int2> itab((size_t)nitem * nbond * nslot, make_int2(0, 0));
  std::vector<int> iD((size_t)nitem * nbond, 0);
  for (int it = 0; it < nitem; ++it)
    for (int b = 0; b <= N; ++b) {
      int2 *row = itab.data() + ((size_t)it * nbond + b) * nslot;
      if (it < M) {
        const auto &m = pb.mps[it];
        int o = 0;
        for (int s = 0; s < nslot; ++s) {
          row[s] = make_int2(o, m.secdim[b][s]);
          o += m.secdim[b][s];
        }
        iD[(size_t)it * nbond + b] = m.dims[b];
      } else {
        const int t = it - M;
        for (int s = 0; s < nslot; ++s) row[s] = kets->hbtab[((size_t)b * kets->n + t) * nslot + s];
        iD[(size_t)it * nbond + b] = kets->htot[(size_t)b * kets->n + t];
      }
    }
  auto idim = [&](int it, int b, int s) { return s < 0 ? 0 : itab[((size_t)it * nbond + b) * nslot + s].y; };
  // largest sector dimensions over the items (block slot sizes)
  std::vector<std::vector<int>> dpad(nbond, std::vector<int>(nslot, 0));
  for (int b = 0; b <= N; ++b) {
    for (int s = 0; s < nslot; ++s)
      for (int it = 0; it < nitem; ++it) dpad[b][s] = std::max(dpad[b][s], idim(it, b, s));
    for (int it = 0; it < nitem; ++it) res.max_pad = std::max(res.max_pad, iD[(size_t)it * nbond + b]);
  }
  // ---- site tensors of every item in the environment precision
  std::vector<const double *> site64((size_t)nitem * N);
  for (int it = 0; it < nitem; ++it)
    for (int p = 0; p < N; ++p)
      site64[(size_t)it * N + p] = it < M ? pb.d_sites + pb.mps[it].site_off[p]
                                          : kets->site_ptr[(size_t)(it - M) * N + p];
  std::vector<const T *> siteT((size_t)nitem * N);
  if (std::is_same<T, double>::value) {
    for (size_t i = 0; i < site64.size(); ++i) siteT[i] = reinterpret_cast<const T *>(site64[i]);
  } else {
    std::vector<int64_t> cnt(site64.size());
    int64_t tot = 0;
    for (int it = 0; it < nitem; ++it)
      for (int p = 0; p < N; ++p) {
        cnt[(size_t)it * N + p] = (int64_t)iD[(size_t)it * nbond + p] * 4 * iD[(size_t)it * nbond + p + 1];
        tot += cnt[(size_t)it * N + p];
      }
    float *buf = c.dev<float>((size_t)tot);
    std::vector<float *> dst(site64.size());
    int64_t o = 0;
    for (size_t i = 0; i < site64.size(); ++i) {
      dst[i] = buf + o;
      o += cnt[i];
      siteT[i] = reinterpret_cast<const T *>(dst[i]);
    }
    launch_cast(c.upload(site64), c.upload(dst), c.upload(cnt), (int)site64.size(), st);
    c.check_launch();
  }
  // ---- block slots and per-site tables
  const MpoDevice &mdev = mpo_dev_for(c, mpo);
  const auto tq1 = Clock::now();
  EnvLayout lay;
  plan_env_layout(mpo, &mdev, N, pb.na, pb.nb, dpad, host_pool(c.ctx), lay);
  // tile mode 2 + k: candidate k on every GEMM list (tests of each shape)
  auto force_tiles = [&](EnvLayout &ly) {
    if (tile_mode < 2) return;
    const int *t = kTileCand[tile_mode - 2];
    for (EnvSiteTabs &tb : ly.tabs) {
      tb.tm1 = tb.tm2 = t[0];
      tb.tn1 = tb.tn2 = t[1];
      for (size_t lv = 0; lv < tb.tmd.size(); ++lv) {
        tb.tmd[lv] = t[0];
        tb.tnd[lv] = t[1];
      }
    }
  };
  force_tiles(lay);
  const std::vector<int64_t> &Lsize = lay.Lsize;
  std::vector<EnvSiteTabs> &tabs = lay.tabs;
  const auto tq2 = Clock::now();
  // ---- algorithmic work with every pair's own block shapes (on a host
  // thread, overlapping the sweeps)
  const double eb = sizeof(T);
  std::thread work_thread([&] {
    double fl[kEnvKinds] = {}, by[kEnvKinds] = {};
    for (const auto &pr : pairs) {
      const int q = (int)(&pr - pairs.data());
      const int bi = pr.first, ki = ket_of_pair[q] < 0 ? pr.first : M + ket_of_pair[q];
      for (int x = 0; x < N; ++x) {
        const EnvSiteTabs &tb = tabs[x];
        for (const EnvG1 &d : tb.g1) {
          const double m = (double)idim(bi, x, d.sbra) * d.nw, k = idim(ki, x, d.s), n = idim(ki, x + 1, d.sk);
          fl[kEnvG1] += 2.0 * m * n * k;
          by[kEnvG1] += eb * (m * k + k * n + m * n);
        }
        for (const MixTask &tk : tb.tasks) {
          const double da = idim(bi, x, tk.sa), db = idim(ki, x + 1, tk.s);
          for (int i = 0; i < tk.nsrc; ++i) {
            fl[kEnvMix] += 2.0 * tb.src_nnz[tk.src0 + i] * da * db;
            by[kEnvMix] += eb * da * tb.srcs[tk.src0 + i].nw_in * db;
          }
          by[kEnvMix] += eb * da * tk.nw_out * db;
        }
        for (const auto &lv : tb.dense)
          for (const EnvGD &d : lv) {
            const double da = idim(bi, x, d.sa), db = idim(ki, x + 1, d.s);
            fl[kEnvDense] += 2.0 * d.nr * d.nc * db * da;
            by[kEnvDense] += eb * ((double)d.nc * db * da + 2.0 * d.nr * db * da);
          }
        for (const EnvG2 &d : tb.g2) {
          const double m = idim(bi, x + 1, d.sbn), n = (double)d.nw * idim(ki, x + 1, d.s);
          for (int g = 0; g < d.nseg; ++g) {
            const double k = idim(bi, x, d.sa[g]);
            fl[kEnvG2] += 2.0 * m * n * k;
            by[kEnvG2] += eb * (k * m + k * n);
          }
          by[kEnvG2] += eb * m * n;
        }
      }
    }
    for (int k = 0; k < kEnvKinds; ++k) {
      res.kind_flops[k] = fl[k];
      res.kind_bytes[k] = by[k];
      res.flops += fl[k];
      res.bytes += by[k];
    }
  });
  struct JoinGuard {
    std::thread &t;
    ~JoinGuard() {
      if (t.joinable()) t.join();
    }
  } join_guard{work_thread};
  // ---- device tables
  require(mpo.site_nnz_off[N] == nnz_total, TNQE_EINVAL, "MPO value layout mismatch");
  // coefficient values in the environment precision for the dense mixing GEMMs
  const T *dvalsT = reinterpret_cast<const T *>(dvals);
  if (!std::is_same<T, double>::value) {
    std::vector<double> h((size_t)nnz_total * M);
    TNQE_HIP(hipMemcpyAsync(h.data(), dvals, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    c.sync();
    std::vector<T> hf(h.begin(), h.end());
    dvalsT = c.upload(hf);
  }
  const int2 *d_itab = c.upload(itab);
  const int *d_iD = c.upload(iD);
  struct DevSite {
    std::vector<EnvGD *> dense;
    EnvG1 *g1;
    EnvG2 *g2;
    MixTask *tasks;
    MixSrc *srcs;
    EnvFinal *fin;
  };
  // sizes of a layout: largest L, X and Y, descriptors (work-list entries per pair)
  struct LaySizes {
    int64_t Lmax = 1, Xmax = 1, Ymax = 1, ndesc = 0;
  };
  auto sizes_of = [&](const EnvLayout &ly) {
    LaySizes z;
    z.Xmax = z.Ymax = 2;   // even: every pair's X and Y start 16-byte aligned
    for (int b = 0; b <= N; ++b) z.Lmax = std::max(z.Lmax, ly.Lsize[b]);
    for (int x = 0; x < N; ++x) {
      z.Xmax = std::max(z.Xmax, ly.tabs[x].Xsize);
      z.Ymax = std::max(z.Ymax, ly.tabs[x].Ysize);
      z.ndesc += (int64_t)ly.tabs[x].g1.size() + ly.tabs[x].tasks.size() + ly.tabs[x].g2.size();
      for (auto &lv : ly.tabs[x].dense) z.ndesc += (int64_t)lv.size();
    }
    return z;
  };
  auto upload_tabs = [&](const EnvLayout &ly) {
    std::vector<DevSite> d(N);
    for (int x = 0; x < N; ++x) {
      d[x].g1 = c.upload(ly.tabs[x].g1);
      d[x].g2 = c.upload(ly.tabs[x].g2);
      d[x].tasks = c.upload(ly.tabs[x].tasks);
      d[x].srcs = c.upload(ly.tabs[x].srcs);
      d[x].fin = c.upload(ly.tabs[x].fin);
      for (auto &lv : ly.tabs[x].dense) d[x].dense.push_back(c.upload(lv));
    }
    return d;
  };
  const double fixed = 256.0 * (5 * N + 24);
  // per pair: the four environment buffers, its entries of the work lists
  // (at most one per descriptor) and its pointer-table entries
  auto per_pair_of = [&](const LaySizes &z) {
    return (double)(2 * z.Lmax + z.Xmax + z.Ymax) * sizeof(T) + (double)z.ndesc * sizeof(EnvWork) +
           (double)(2 * N + 12) * sizeof(void *);
  };
  const LaySizes gz = sizes_of(lay);
  const int npair = (int)pairs.size();
  const double per_pair = per_pair_of(gz);
  double budget = 96.0 * (1ull << 30);
  // a caller's workspace too small for one pair in the common layout: every
  // pair runs alone, in a layout of its own two items' dimensions
  bool own_layouts = false;
  if (c.ctx->pool.arena()) {
    budget = std::min(budget, (double)c.ctx->pool.available() - fixed);
    own_layouts = budget < per_pair;
  }
  std::vector<DevSite> ds;
  if (!own_layouts) ds = upload_tabs(lay);
  c.sync();
  const auto tq3 = Clock::now();
  double t_work = 0.0, t_launch = 0.0, t_wait = 0.0;
  // ---- pair batches under a memory budget
  const int batch = own_layouts ? 1 : std::max(1, std::min(npair, (int)(budget / std::max(1.0, per_pair))));
  res.H.assign(npair, 0.0);
  res.S.assign(npair, 0.0);
  hipEvent_t e0 = c.ctx->ev[0], e1 = c.ctx->ev[1];
  EnvLayout own;
  for (int p0 = 0; p0 < npair; p0 += batch) {
    const int nb_ = std::min(batch, npair - p0);
    const size_t mk = c.ctx->pool.mark();
    const EnvLayout *cur = &lay;
    LaySizes z = gz;
    std::vector<DevSite> ds_own;
    if (own_layouts) {
      const int bi = pairs[p0].first, ki = ket_of_pair[p0] < 0 ? bi : M + ket_of_pair[p0];
      std::vector<std::vector<int>> dq(nbond, std::vector<int>(nslot, 0));
      for (int b = 0; b <= N; ++b)
        for (int s2 = 0; s2 < nslot; ++s2) dq[b][s2] = std::max(idim(bi, b, s2), idim(ki, b, s2));
      plan_env_layout(mpo, &mdev, N, pb.na, pb.nb, dq, host_pool(c.ctx), own);
      force_tiles(own);
      cur = &own;
      z = sizes_of(own);
      require(per_pair_of(z) <= (double)c.ctx->pool.available() - fixed - 64.0 * (z.ndesc + 64), TNQE_EWORKSPACE,
              "workspace too small for the environment sweep of one pair (" +
                  std::to_string((int64_t)per_pair_of(z)) + " bytes needed, " +
                  std::to_string(c.ctx->pool.available()) + " left)");
      ds_own = upload_tabs(own);
    }
    const std::vector<EnvSiteTabs> &ctabs = cur->tabs;
    const std::vector<DevSite> &cds = own_layouts ? ds_own : ds;
    const int64_t Lmax = z.Lmax, Xmax = z.Xmax, Ymax = z.Ymax;
    T *bufL0 = c.dev<T>((size_t)Lmax * nb_), *bufL1 = c.dev<T>((size_t)Lmax * nb_);
    T *bufX = c.dev<T>((size_t)Xmax * nb_), *bufY = c.dev<T>((size_t)Ymax * nb_);
    std::vector<T *> L0(nb_), L1(nb_), X(nb_), Y(nb_);
    std::vector<int> basis(nb_), bra_item(nb_), ket_item(nb_);
    for (int q = 0; q < nb_; ++q) {
      L0[q] = bufL0 + (size_t)q * Lmax;
      L1[q] = bufL1 + (size_t)q * Lmax;
      X[q] = bufX + (size_t)q * Xmax;
      Y[q] = bufY + (size_t)q * Ymax;
      const int i = pairs[p0 + q].first;
      basis[q] = i;
      bra_item[q] = i;
      ket_item[q] = ket_of_pair[p0 + q] < 0 ? i : M + ket_of_pair[p0 + q];
    }
    T **dL0 = c.upload(L0), **dL1 = c.upload(L1), **dX = c.upload(X), **dY = c.upload(Y);
    const int *dbasis = c.upload(basis);
    EnvGeom geom{d_itab, d_iD, c.upload(bra_item), c.upload(ket_item), nbond, nslot};
    std::vector<const T *> vptr(nb_);
    for (int q = 0; q < nb_; ++q) vptr[q] = dvalsT + (size_t)basis[q] * nnz_total;
    const T *const *dvptr = c.upload(vptr);
    std::vector<const T *const *> dbra(N), dket(N);
    for (int x = 0; x < N; ++x) {
      std::vector<const T *> bp(nb_), kp(nb_);
      for (int q = 0; q < nb_; ++q) {
        bp[q] = siteT[(size_t)bra_item[q] * N + x];
        kp[q] = siteT[(size_t)ket_item[q] * N + x];
      }
      dbra[x] = c.upload(bp);
      dket[x] = c.upload(kp);
    }
    // autotuning (first batch, common layout): each environment GEMM list
    // whose shape class has no tuned tile yet is timed with every tile shape
    // on this batch's buffers (their contents are not used yet: the real
    // sweep overwrites every output afterwards); the fastest is kept
    if (tile_mode == 1 && p0 == 0 && !own_layouts) {
      const auto tt0 = Clock::now();
      load_tiles(c.ctx);
      auto tiles = [](int64_t Mm, int64_t Nn, int tm, int tn) {
        return (Mm <= 0 || Nn <= 0) ? (int64_t)0 : ((Mm + tm - 1) / tm) * ((Nn + tn - 1) / tn);
      };
      bool added = false;
      for (int x = 0; x < N; ++x)
        for (int kind = 0; kind < 2; ++kind) {
          if (kind == 1 && x == N - 1) continue;
          EnvSiteTabs &tb = lay.tabs[x];
          const int nd = kind == 0 ? (int)tb.g1.size() : (int)tb.g2.size();
          if (nd == 0) continue;
          auto extent = [&](int di, int q, int64_t &Mm, int64_t &Nn) {
            if (kind == 0) {
              const EnvG1 &d = tb.g1[di];
              Mm = (int64_t)idim(bra_item[q], x, d.sbra) * d.nw;
              Nn = idim(ket_item[q], x + 1, d.sk);
            } else {
              const EnvG2 &d = tb.g2[di];
              Mm = idim(bra_item[q], x + 1, d.sbn);
              Nn = (int64_t)d.nw * idim(ket_item[q], x + 1, d.s);
            }
          };
          int64_t maxM = 1, maxN = 1;
          double work = 1.0;
          for (int di = 0; di < nd; ++di)
            for (int q = 0; q < nb_; ++q) {
              int64_t Mm, Nn;
              extent(di, q, Mm, Nn);
              maxM = std::max(maxM, Mm);
              maxN = std::max(maxN, Nn);
              work += (double)Mm * Nn;
            }
          const std::array<int, 5> key = {kind, (int)sizeof(T) + 100 * cm, ceil_log2((double)maxM),
                                          ceil_log2((double)maxN), ceil_log2(work)};
          auto it = c.ctx->tiles.find(key);
          if (it == c.ctx->tiles.end()) {
            float best = 1e30f;
            std::pair<int, int> pick = {64, 64};
            for (const auto &cd : kTileCand) {
              // pair-major, as the sweep's own lists
              std::vector<EnvWork> list;
              int nwg = 0;
              for (int q = 0; q < nb_; ++q)
                for (int di = 0; di < nd; ++di) {
                  int64_t Mm, Nn;
                  extent(di, q, Mm, Nn);
                  const int64_t cnt = tiles(Mm, Nn, cd[0], cd[1]);
                  if (cnt <= 0) continue;
                  require(nwg + cnt < (int64_t)1 << 31, TNQE_ESHAPE, "environment launch exceeds the grid limit");
                  list.push_back(EnvWork{di, q, nwg});
                  nwg += (int)cnt;
                }
              const EnvWork *dl = c.upload(list);
              auto launch = [&] {
                if (kind == 0)
                  launch_env_g1<T>(ds[x].g1, dl, (int)list.size(), nwg, cd[0], cd[1], geom, dL0, dket[x], dX, st, cm);
                else
                  launch_env_g2<T>(ds[x].g2, dl, (int)list.size(), nwg, cd[0], cd[1], geom, dbra[x], dY, dL1, st, cm);
              };
              launch();
              TNQE_HIP(hipEventRecord(e0, st));
              for (int rep = 0; rep < 3; ++rep) launch();
              TNQE_HIP(hipEventRecord(e1, st));
              c.check_launch();
              TNQE_HIP(hipEventSynchronize(e1));
              float ms = 0.0f;
              TNQE_HIP(hipEventElapsedTime(&ms, e0, e1));
              if (ms < best) {
                best = ms;
                pick = {cd[0], cd[1]};
              }
            }
            it = c.ctx->tiles.emplace(key, pick).first;
            added = true;
          }
          if (kind == 0) {
            tb.tm1 = it->second.first;
            tb.tn1 = it->second.second;
          } else {
            tb.tm2 = it->second.first;
            tb.tn2 = it->second.second;
          }
        }
      c.sync();
      if (added) save_tiles(c.ctx);
      res.tune_ms += ms_since(tt0);
    }
    const auto tb0 = Clock::now();
    // work lists of the batch: only the tiles (chunks) inside every pair's
    // own extents; sites in parallel on the host workers
    struct SiteWork {
      std::vector<EnvWork> g1, mix, mix2, g2;
      std::vector<std::vector<EnvWork>> dense;
      int n1 = 0, nmix = 0, nmix2 = 0, n2 = 0;
      std::vector<int> nd;
    };
    std::vector<SiteWork> sw(N);
    host_pool(c.ctx).parallel_for(N, [&](int x) {
      const EnvSiteTabs &tb = ctabs[x];
      SiteWork &w = sw[x];
      auto add = [](std::vector<EnvWork> &list, int &nwg, int desc, int q, int64_t cnt) {
        if (cnt <= 0) return;
        require(nwg + cnt < (int64_t)1 << 31, TNQE_ESHAPE, "environment launch exceeds the grid limit");
        list.push_back(EnvWork{desc, q, nwg});
        nwg += (int)cnt;
      };
      auto tiles = [](int64_t M, int64_t Nn, int tm, int tn) {
        return (M <= 0 || Nn <= 0) ? (int64_t)0 : ((M + tm - 1) / tm) * ((Nn + tn - 1) / tn);
      };
      // pair-major order: the problems of one pair, which share their
      // operand blocks, run close together in time and reuse them from L2
      for (int q = 0; q < nb_; ++q)
        for (size_t di = 0; di < tb.g1.size(); ++di) {
          const EnvG1 &d = tb.g1[di];
          add(w.g1, w.n1, (int)di, q,
              tiles((int64_t)idim(bra_item[q], x, d.sbra) * d.nw, idim(ket_item[q], x + 1, d.sk), tb.tm1, tb.tn1));
        }
      // channel mix: blocks of an even number of ket columns take the kernel
      // that loads column pairs as one vector (all X and Y offsets are even)
      for (int q = 0; q < nb_; ++q)
        for (size_t ti = 0; ti < tb.tasks.size(); ++ti) {
          const MixTask &tk = tb.tasks[ti];
          const int da = idim(bra_item[q], x, tk.sa), db = idim(ket_item[q], x + 1, tk.s);
          if (db % 2 == 0) {
            const int64_t items = (int64_t)((da + kMix2Rows - 1) / kMix2Rows) * tk.nw_out * (db / 2);
            add(w.mix2, w.nmix2, (int)ti, q, (items + 255) / 256);
            continue;
          }
          const int64_t items =
              (int64_t)((da + kMixRows - 1) / kMixRows) * tk.nw_out * ((db + kMixCols - 1) / kMixCols);
          add(w.mix, w.nmix, (int)ti, q, (items + 255) / 256);
        }
      w.dense.resize(tb.dense.size());
      w.nd.assign(tb.dense.size(), 0);
      for (size_t lv = 0; lv < tb.dense.size(); ++lv)
        for (int q = 0; q < nb_; ++q)
          for (size_t di = 0; di < tb.dense[lv].size(); ++di) {
            const EnvGD &d = tb.dense[lv][di];
            add(w.dense[lv], w.nd[lv], (int)di, q,
                tiles(d.nr, (int64_t)idim(bra_item[q], x, d.sa) * idim(ket_item[q], x + 1, d.s), tb.tmd[lv],
                      tb.tnd[lv]));
          }
      for (int q = 0; q < nb_; ++q)
        for (size_t di = 0; di < tb.g2.size(); ++di) {
          const EnvG2 &d = tb.g2[di];
          add(w.g2, w.n2, (int)di, q,
              tiles(idim(bra_item[q], x + 1, d.sbn), (int64_t)d.nw * idim(ket_item[q], x + 1, d.s), tb.tm2,
                    tb.tn2));
        }
    });
    struct DevWork {
      const EnvWork *g1, *mix, *mix2, *g2;
      std::vector<const EnvWork *> dense;
    };
    std::vector<DevWork> dw(N);
    for (int x = 0; x < N; ++x) {
      dw[x].g1 = c.upload(sw[x].g1);
      dw[x].mix = c.upload(sw[x].mix);
      dw[x].mix2 = c.upload(sw[x].mix2);
      dw[x].g2 = c.upload(sw[x].g2);
      for (auto &lv : sw[x].dense) dw[x].dense.push_back(c.upload(lv));
    }
    const auto tb1 = Clock::now();
    t_work += ms_between(tb0, tb1);
    std::vector<const double *> bra64(nb_);
    for (int q = 0; q < nb_; ++q) bra64[q] = site64[(size_t)bra_item[q] * N + N - 1];
    const double *const *dbra64 = c.upload(bra64);
    double *dout = c.dev<double>((size_t)nb_ * 2);
    // one event between consecutive launches: launch i runs from tick i to i + 1
    std::vector<int> tick_kind;
    // per-launch timing needs one event per launch; a call that must not
    // allocate uses only the events the context already has, else none
    size_t nticks = 1;
    for (int x = 0; x < N; ++x) nticks += 2 + ctabs[x].dense.size() + 1;
    const bool timed = !c.ctx->no_alloc || nticks <= c.ctx->env_ev.size();
    auto tick = [&](int kind) {
      if (!timed) return;
      const size_t i = tick_kind.size();
      if (i >= c.ctx->env_ev.size()) {
        hipEvent_t e;
        TNQE_HIP(hipEventCreate(&e));
        c.ctx->env_ev.push_back(e);
      }
      TNQE_HIP(hipEventRecord(c.ctx->env_ev[i], st));
      tick_kind.push_back(kind);
    };
    TNQE_HIP(hipEventRecord(e0, st));
    launch_env_init<T>(dL0, nb_, cur->Lsize[0], st);
    T **Lc = dL0, **Ln = dL1;
    for (int x = 0; x < N; ++x) {
      const EnvSiteTabs &tb = ctabs[x];
      const SiteWork &w = sw[x];
      tick(kEnvG1);
      launch_env_g1<T>(cds[x].g1, dw[x].g1, (int)w.g1.size(), w.n1, tb.tm1, tb.tn1, geom, Lc, dket[x], dX, st, cm);
      MixArgs ma{};
      ma.tasks = cds[x].tasks;
      ma.work = dw[x].mix;
      ma.nwork = (int)w.mix.size();
      ma.nchunk = w.nmix;
      ma.srcs = cds[x].srcs;
      ma.rowptr = mdev.rowptr;
      ma.col = mdev.col;
      ma.vals = dvals;
      ma.basis_stride = nnz_total;
      ma.basis = dbasis;
      tick(kEnvMix);
      launch_mix<T>(ma, geom, dX, dY, st);
      MixArgs m2 = ma;
      m2.work = dw[x].mix2;
      m2.nwork = (int)w.mix2.size();
      m2.nchunk = w.nmix2;
      launch_mix2<T>(m2, geom, dX, dY, st);
      for (size_t lv = 0; lv < tb.dense.size(); ++lv) {
        tick(kEnvDense);
        launch_env_gd<T>(cds[x].dense[lv], dw[x].dense[lv], (int)w.dense[lv].size(), w.nd[lv], tb.tmd[lv],
                         tb.tnd[lv], geom, dvptr, dX, dY, st, cm);
      }
      if (x < N - 1) {
        tick(kEnvG2);
        launch_env_g2<T>(cds[x].g2, dw[x].g2, (int)w.g2.size(), w.n2, tb.tm2, tb.tn2, geom, dbra[x], dY, Ln, st, cm);
        std::swap(Lc, Ln);
      } else {
        tick(kEnvFinal);
        launch_env_final<T>(geom, x, dbra64, dY, cds[x].fin, (int)tb.fin.size(), 2, dout, nb_, st);
      }
      c.check_launch();
    }
    tick(-1);
    TNQE_HIP(hipEventRecord(e1, st));
    std::vector<double> out((size_t)nb_ * 2);
    TNQE_HIP(hipMemcpyAsync(out.data(), dout, out.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    const auto tb2 = Clock::now();
    t_launch += ms_between(tb1, tb2);
    c.sync();
    t_wait += ms_between(tb2, Clock::now());
    float ms = 0.0f;
    TNQE_HIP(hipEventElapsedTime(&ms, e0, e1));
    res.kernel_ms += ms;
    for (size_t i = 0; i + 1 < tick_kind.size(); ++i) {
      float t = 0.0f;
      TNQE_HIP(hipEventElapsedTime(&t, c.ctx->env_ev[i], c.ctx->env_ev[i + 1]));
      res.kind_ms[tick_kind[i]] += t;
      res.kind_launches[tick_kind[i]]++;
    }
    for (int q = 0; q < nb_; ++q) {
      res.H[p0 + q] = out[(size_t)q * 2 + mpo.final_H];
      res.S[p0 + q] = out[(size_t)q * 2 + mpo.final_I];
    }
    c.ctx->pool.rewind(mk);
  }
  if (debug_timing()) {
    double mb[6] = {};
    for (int x = 0; x < N; ++x) {
      mb[0] += tabs[x].g1.size() * sizeof(EnvG1) / 1e6;
      mb[1] += tabs[x].g2.size() * sizeof(EnvG2) / 1e6;
      mb[2] += tabs[x].tasks.size() * sizeof(MixTask) / 1e6;
      mb[3] += tabs[x].srcs.size() * sizeof(MixSrc) / 1e6;
      for (auto &lv : tabs[x].dense) mb[5] += lv.size() * sizeof(EnvGD) / 1e6;
    }
    std::fprintf(stderr,
                 "env phase host: items %.1f ms, site tables %.1f ms, device tables %.1f ms (MB: g1 %.1f g2 %.1f "
                 "tasks %.1f sources %.1f dense %.1f), work lists %.1f ms, launches %.1f ms, wait %.1f ms\n",
                 ms_between(tq0, tq1), ms_between(tq1, tq2), ms_between(tq2, tq3), mb[0], mb[1], mb[2], mb[3], mb[5],
                 t_work, t_launch, t_wait);
  }
}

// ------------------------------------------------------------ one solve
struct SolveOut {
  std::vector<double> H, S;
  double E = 0.0;
  std::vector<double> c;
  tnqe_report rep{};
  int status = 0;
};

// rotated integrals h^(i) = U^T h U, (pq|rs)^(i)
void rotate_integrals(const tnqe_problem &pb, const std::vector<double> &U, std::vector<double> &hi,
                      std::vector<double> &gi) {
  const int N = pb.N;
  const size_t N2 = (size_t)N * N;
  auto rot2 = [&](const double *A, double *out) {   // out = U^T A U
    std::vector<double> t(N2, 0.0);
    for (int p = 0; p < N; ++p)
      for (int b = 0; b < N; ++b) {
        double acc = 0.0;
        for (int q = 0; q < N; ++q) acc += A[p * N + q] * U[q * N + b];
        t[p * N + b] = acc;
      }
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) {
        double acc = 0.0;
        for (int p = 0; p < N; ++p) acc += U[p * N + a] * t[p * N + b];
        out[a * N + b] = acc;
      }
  };
  hi.assign(N2, 0.0);
  rot2(pb.h.data(), hi.data());
  gi.assign(N2 * N2, 0.0);
  if (pb.K > 0) {
    // (pq|rs) = sum_k L^k_pq L^k_rs is symmetric under pq <-> rs: the upper
    // triangle is accumulated (in the same k order) and mirrored
    std::vector<double> Lk(N2);
    for (int k = 0; k < pb.K; ++k) {
      rot2(pb.L.data() + (size_t)k * N2, Lk.data());
      for (size_t x = 0; x < N2; ++x) {
        const double v = Lk[x];
        if (v == 0.0) continue;
        double *row = gi.data() + x * N2;
        for (size_t y = x; y < N2; ++y) row[y] += v * Lk[y];
      }
    }
    for (size_t x = 0; x < N2; ++x)
      for (size_t y = x + 1; y < N2; ++y) gi[y * N2 + x] = gi[x * N2 + y];
  } else {
    // four quarter transformations of (pq|rs)
    std::vector<double> a(pb.g), b(N2 * N2);
    for (int pass = 0; pass < 4; ++pass) {
      // contract the first index with U and rotate the index order (pqrs -> qrsP)
      for (int P = 0; P < N; ++P)
        for (size_t rest = 0; rest < N2 * N; ++rest) {
          double acc = 0.0;
          for (int p = 0; p < N; ++p) acc += U[p * N + P] * a[(size_t)p * N2 * N + rest];
          b[rest * N + P] = acc;
        }
      std::swap(a, b);
    }
    gi = a;
  }
}

MpoStructure &mpo_for(tnqe_ctx *ctx, int N) {
  auto it = ctx->mpo_cache.find(N);
  if (it != ctx->mpo_cache.end()) return *it->second;
  auto m = std::make_unique<MpoStructure>();
  mpo_build_structure(N, *m);
  MpoStructure &ref = *m;
  ctx->mpo_cache[N] = std::move(m);
  return ref;
}

// Capacity of every bond of a rotated ket: the largest input dimension, or
// min(chi, exact dimension of the (n_alpha, n_beta) sector bond) if larger.
std::vector<int> bond_caps(const tnqe_problem &pb, int chi_cap) {
  const int N = pb.N;
  std::vector<int> cap(N + 1, 1);
  for (int b = 0; b <= N; ++b) {
    double ex = 0.0;
    const int a0 = std::max(0, pb.na - (N - b)), a1 = std::min(b, pb.na);
    const int b0 = std::max(0, pb.nb - (N - b)), b1 = std::min(b, pb.nb);
    for (int a = a0; a <= a1; ++a)
      for (int bb = b0; bb <= b1; ++bb)
        ex += std::min(binom(b, a) * binom(b, bb), binom(N - b, pb.na - a) * binom(N - b, pb.nb - bb));
    int mx = 0;
    for (int i = 0; i < pb.M; ++i) mx = std::max(mx, pb.mps[i].dims[b]);
    cap[b] = std::max(mx, (int)std::min<double>(ex, (double)chi_cap));
  }
  return cap;
}

// The Givens networks of the (basis i, ket j) pairs offd (j != i), all in
// lock step: canon receives left-canonical copies of all M MPS (centre on the
// last site) and kets[t] the MPS offd[t].second taken into basis
// offd[t].first, truncated after every gate (App. A1, App. A3, Sec. II.B).
void gate_phase(Call &c, tnqe_problem &pb, const std::vector<std::pair<int, int>> &offd, int chi_cap,
                const tnqe_options &op, int max_sweeps, KetSet &canon, KetSet &kets, TruncStats &ts) {
  tnqe_ctx *ctx = c.ctx;
  const int N = pb.N, M = pb.M, nslot = pb.nslot();
  const int P = (int)offd.size();
  std::vector<std::vector<int>> gpos(P);
  std::vector<std::vector<double>> gth(P);
  std::vector<int> dsign(P, 1);
  host_pool(ctx).parallel_for(P, [&](int t) {
    const auto &Ui = pb.mps[offd[t].first].U, &Uj = pb.mps[offd[t].second].U;
    std::vector<double> W((size_t)N * N, 0.0);
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) {
        double acc = 0.0;
        for (int p = 0; p < N; ++p) acc += Ui[p * N + a] * Uj[p * N + b];
        W[a * N + b] = acc;
      }
    givens_plan(N, W.data(), gpos[t], gth[t], dsign[t]);
  });
  ts.discarded.assign(P, 0.0);
  {
    const std::vector<int> cap = bond_caps(pb, chi_cap);
    // left-canonical copies of every MPS used as a ket
    canon.init(&c, M, N, pb.na, pb.nb, cap);
    {
      std::vector<double *> dst(M), src(M);
      std::vector<int64_t> cnt(M);
      for (int p = 0; p < N; ++p) {
        for (int i = 0; i < M; ++i) {
          dst[i] = canon.site_ptr[(size_t)i * N + p];
          src[i] = pb.d_sites + pb.mps[i].site_off[p];
          cnt[i] = (int64_t)pb.mps[i].dims[p] * 4 * pb.mps[i].dims[p + 1];
        }
        const size_t mk = ctx->pool.mark();
        launch_copy(c.upload(dst), c.upload(src), c.upload(cnt), M, ctx->stream);
        c.sync();
        ctx->pool.rewind(mk);
      }
      for (int b = 0; b <= N; ++b) {
        for (int i = 0; i < M; ++i)
          for (int s = 0; s < nslot; ++s) canon.dim(b, i, s) = pb.mps[i].secdim[b][s];
        canon.commit_bond(b);
      }
      for (int p = 0; p + 1 < N; ++p) {
        const size_t mk = ctx->pool.mark();
        move_right(canon, p, max_sweeps, &ts.svd);
        c.sync();
        ctx->pool.rewind(mk);
      }
    }
    if (P == 0) {
      c.sync();
      return;
    }
    kets.init(&c, P, N, pb.na, pb.nb, cap);
    {
      std::vector<double *> dst(P), src(P);
      std::vector<int64_t> cnt(P);
      for (int p = 0; p < N; ++p) {
        for (int t = 0; t < P; ++t) {
          const int j = offd[t].second;
          dst[t] = kets.site_ptr[(size_t)t * N + p];
          src[t] = canon.site_ptr[(size_t)j * N + p];
          cnt[t] = (int64_t)canon.htot[(size_t)p * M + j] * 4 * canon.htot[(size_t)(p + 1) * M + j];
        }
        const size_t mk = ctx->pool.mark();
        launch_copy(c.upload(dst), c.upload(src), c.upload(cnt), P, ctx->stream);
        c.sync();
        ctx->pool.rewind(mk);
      }
      for (int b = 0; b <= N; ++b) {
        for (int t = 0; t < P; ++t)
          for (int s = 0; s < nslot; ++s) kets.dim(b, t, s) = canon.dim(b, offd[t].second, s);
        kets.commit_bond(b);
      }
      // parity gate on the last site where det(U_i^T U_j) = -1
      std::vector<double *> sg;
      std::vector<int> rows;
      for (int t = 0; t < P; ++t)
        if (dsign[t] < 0) {
          sg.push_back(kets.site_ptr[(size_t)t * N + N - 1]);
          rows.push_back(kets.htot[(size_t)(N - 1) * P + t]);
        }
      if (!sg.empty()) launch_site_sign(c.upload(sg), c.upload(rows), (int)sg.size(), 1, ctx->stream);
      c.sync();
    }
    int centre = N - 1;
    const size_t ngate = gpos[0].size();
    std::vector<double> gates((size_t)P * 2);   // (cos, sin) of every pair's angle
    Clock::time_point t_prev_end = Clock::now();
    for (size_t g = 0; g < ngate; ++g) {
      const int a = gpos[0][g];
      // a gate of angle 0 for every pair is the identity; while no pair's
      // bond a+1 exceeds chi its truncation could only drop weight below the
      // tau_w cut, so it is not applied (no network at all for unrotated MPS)
      bool identity = true;
      for (int t = 0; t < P; ++t) {
        require(gpos[t][g] == a, TNQE_EINVAL, "gate positions differ between pairs");
        identity = identity && gth[t][g] == 0.0 && kets.htot[(size_t)(a + 1) * P + t] <= chi_cap;
      }
      if (identity) continue;
      const size_t mk = ctx->pool.mark();
      const auto tm0 = Clock::now();
      // each move's scratch goes back before the next move
      const auto tmv = Clock::now();
      while (centre > a) {
        const size_t mm = ctx->pool.mark();
        move_left(kets, centre, max_sweeps, &ts.svd);
        ctx->pool.rewind(mm);
        --centre;
      }
      while (centre < a) {
        const size_t mm = ctx->pool.mark();
        move_right(kets, centre, max_sweeps, &ts.svd);
        ctx->pool.rewind(mm);
        ++centre;
      }
      ts.move_wall_ms += ms_since(tmv);
      const auto tm1 = Clock::now();
      if (debug_timing() && g > 0) g_gate_timing.caller_ms += ms_between(t_prev_end, tm0);
      for (int t = 0; t < P; ++t) {
        gates[2 * t] = std::cos(gth[t][g]);
        gates[2 * t + 1] = std::sin(gth[t][g]);
      }
      gate_step(kets, a, gates, chi_cap, op.tau_w, max_sweeps, op.renormalize != 0, ts);
      centre = a + 1;
      ctx->pool.rewind(mk);
      if (debug_timing()) {
        g_gate_timing.move_ms += std::chrono::duration<double, std::milli>(tm1 - tm0).count();
        g_gate_timing.step_ms += std::chrono::duration<double, std::milli>(Clock::now() - tm1).count();
        t_prev_end = Clock::now();
      }
    }
    c.sync();
    ts.svd.collect(ctx);
    if (debug_timing()) {
      std::fprintf(stderr,
                   "gate phase host: %d steps, move %.1f ms, gate step %.1f ms (build %.1f [parallel %.1f], "
                   "two-site %.1f, svd launches %.1f, sync wait %.1f, selection %.1f, split %.1f), between "
                   "steps %.1f\n",
                   g_gate_timing.steps, g_gate_timing.move_ms, g_gate_timing.step_ms, g_gate_timing.build_ms,
                   g_gate_timing.plan_par_ms, g_gate_timing.two_site_ms, g_gate_timing.svd_host_ms,
                   g_gate_timing.sync_ms, g_gate_timing.select_ms, g_gate_timing.post_ms, g_gate_timing.caller_ms);
      g_gate_timing = GateHostTiming{};
    }
  }
}

void solve_one(tnqe_ctx *ctx, tnqe_problem &pb, const tnqe_options &op, SolveOut &out) {
  Call c{ctx};
  const auto t0 = Clock::now();
  const int N = pb.N, M = pb.M, nslot = pb.nslot();
  const int chi_cap = op.chi_cap_override > 0 ? op.chi_cap_override : op.chi;
  require(chi_cap >= 1, TNQE_EINVAL, "chi must be >= 1");
  const int max_sweeps = op.max_sweeps > 0 ? op.max_sweeps : 40;
  tnqe_report &rep = out.rep;
  rep = tnqe_report{};
  // ---- host: integrals, MPO, plans
  MpoStructure &mpo = mpo_for(ctx, N);
  const int64_t nnz = mpo.site_nnz_off[N];
  // the coefficients of all bases go straight into pinned staging memory
  double *vals = static_cast<double *>(ctx->staging.reserve((size_t)nnz * M * sizeof(double)));
  {
    // one basis per host thread: rotated integrals and MPO coefficients
    const int nth = std::max(1, std::min<int>(M, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    std::vector<std::string> errs(nth);
    for (int w = 0; w < nth; ++w)
      pool.emplace_back([&, w] {
        try {
          std::vector<double> slotv, v1, hi, gi;
          for (int i = w; i < M; i += nth) {
            rotate_integrals(pb, pb.mps[i].U, hi, gi);
            mpo_values(mpo, hi.data(), gi.data(), v1, slotv);
            std::copy(v1.begin(), v1.end(), vals + (size_t)i * nnz);
          }
        } catch (const std::exception &e) {
          errs[w] = e.what();
        }
      });
    for (auto &t : pool) t.join();
    for (auto &e : errs) require(e.empty(), TNQE_EINVAL, e);
  }
  double *dvals = c.dev<double>((size_t)nnz * M);
  TNQE_HIP(hipMemcpyAsync(dvals, vals, (size_t)nnz * M * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  std::vector<std::pair<int, int>> pairs;
  std::vector<int> ket_of_pair;
  std::vector<std::pair<int, int>> offd;
  for (int i = 0; i < M; ++i)
    for (int j = i; j < M; ++j) {
      pairs.push_back({i, j});
      if (i == j) {
        ket_of_pair.push_back(-1);
      } else {
        ket_of_pair.push_back((int)offd.size());
        offd.push_back({i, j});
      }
    }
  const int P = (int)offd.size();
  rep.t_host_ms = ms_since(t0);
  // ---- gate phase
  const auto tg = Clock::now();
  KetSet canon, kets;
  TruncStats ts;
  if (P > 0) gate_phase(c, pb, offd, chi_cap, op, max_sweeps, canon, kets, ts);
  rep.t_gates_ms = ms_since(tg);
  // ---- environment sweep
  const auto te = Clock::now();
  EnvResult er;
  double shift_total = 0.0;   // c N_e of the shifted FP32 mode
  if (op.precision == TNQE_ENV_FP32) {
    env_phase<float>(c, pb, P > 0 ? &kets : nullptr, pairs, ket_of_pair, mpo, dvals, nnz, er, op.autotune);
    rep.n_fp32_pairs = (int)pairs.size();
  } else if (op.precision == TNQE_ENV_FP32_SHIFT || op.precision == TNQE_ENV_BF16 ||
             op.precision == TNQE_ENV_BF16X3) {
    const int cm = op.precision == TNQE_ENV_BF16 ? 1 : op.precision == TNQE_ENV_BF16X3 ? 2 : 0;
    // reference energy: the FP64 element of pair (0, 0)
    {
      EnvResult e0;
      const size_t me = ctx->pool.mark();
      const std::vector<std::pair<int, int>> p0 = {{0, 0}};
      const std::vector<int> k0 = {-1};
      env_phase<double>(c, pb, P > 0 ? &kets : nullptr, p0, k0, mpo, dvals, nnz, e0, op.autotune);
      c.sync();
      ctx->pool.rewind(me);
      shift_total = e0.H[0];
    }
    // coefficients of H - c N in every basis: the one-electron diagonal moves
    // by -c (the basis change is orthogonal, so the same c in every basis);
    // the coefficient map is affine in (h, g), so the move is c times the
    // values of (h = 1, g = 0) minus those of (0, 0)
    const int ne = pb.na + pb.nb;
    const double cpe = ne > 0 ? shift_total / ne : 0.0;
    if (ne == 0) shift_total = 0.0;
    std::vector<double> hI((size_t)N * N, 0.0), h0((size_t)N * N, 0.0), g0((size_t)N * N * N * N, 0.0), vI, v0, sv;
    for (int p = 0; p < N; ++p) hI[(size_t)p * N + p] = 1.0;
    mpo_values(mpo, hI.data(), g0.data(), vI, sv);
    mpo_values(mpo, h0.data(), g0.data(), v0, sv);
    for (size_t j = 0; j < vI.size(); ++j) vI[j] -= v0[j];
    double *dvs = c.dev<double>((size_t)nnz * M);
    launch_shift_vals(dvals, c.upload(vI), -cpe, nnz, M, dvs, ctx->stream);
    c.check_launch();
    env_phase<float>(c, pb, P > 0 ? &kets : nullptr, pairs, ket_of_pair, mpo, dvs, nnz, er, op.autotune, cm);
    rep.n_fp32_pairs = (int)pairs.size();
  } else if (op.precision == TNQE_ENV_MIXED) {
    // FP32 for pairs whose rotated ket kept at most kMixedNorm2 of its squared
    // norm (1 - summed discarded weight), FP64 for the rest
    constexpr double kMixedNorm2 = 1e-6;
    std::vector<std::pair<int, int>> p64, p32;
    std::vector<int> k64, k32, q64, q32;
    for (size_t q = 0; q < pairs.size(); ++q) {
      const int t = ket_of_pair[q];
      if (t >= 0 && 1.0 - ts.discarded[t] <= kMixedNorm2) {
        p32.push_back(pairs[q]);
        k32.push_back(t);
        q32.push_back((int)q);
      } else {
        p64.push_back(pairs[q]);
        k64.push_back(t);
        q64.push_back((int)q);
      }
    }
    EnvResult e64, e32;
    const size_t me = ctx->pool.mark();
    if (!p64.empty()) env_phase<double>(c, pb, P > 0 ? &kets : nullptr, p64, k64, mpo, dvals, nnz, e64, op.autotune);
    c.sync();
    ctx->pool.rewind(me);
    if (!p32.empty()) env_phase<float>(c, pb, P > 0 ? &kets : nullptr, p32, k32, mpo, dvals, nnz, e32, op.autotune);
    er.H.assign(pairs.size(), 0.0);
    er.S.assign(pairs.size(), 0.0);
    for (size_t q = 0; q < q64.size(); ++q) {
      er.H[q64[q]] = e64.H[q];
      er.S[q64[q]] = e64.S[q];
    }
    for (size_t q = 0; q < q32.size(); ++q) {
      er.H[q32[q]] = e32.H[q];
      er.S[q32[q]] = e32.S[q];
    }
    er.flops = e64.flops + e32.flops;
    er.tune_ms = e64.tune_ms + e32.tune_ms;
    er.bytes = e64.bytes + e32.bytes;
    er.kernel_ms = e64.kernel_ms + e32.kernel_ms;
    er.max_pad = std::max(e64.max_pad, e32.max_pad);
    for (int k = 0; k < kEnvKinds; ++k) {
      er.kind_ms[k] = e64.kind_ms[k] + e32.kind_ms[k];
      er.kind_flops[k] = e64.kind_flops[k] + e32.kind_flops[k];
      er.kind_bytes[k] = e64.kind_bytes[k] + e32.kind_bytes[k];
      er.kind_launches[k] = e64.kind_launches[k] + e32.kind_launches[k];
    }
    rep.n_fp32_pairs = (int)p32.size();
  } else {
    env_phase<double>(c, pb, P > 0 ? &kets : nullptr, pairs, ket_of_pair, mpo, dvals, nnz, er, op.autotune);
  }
  rep.t_env_ms = ms_since(te);
  // ---- pencil and eigensolve
  const auto tq = Clock::now();
  out.H.assign((size_t)M * M, 0.0);
  out.S.assign((size_t)M * M, 0.0);
  // the eigenproblem runs on the pencil as computed (shifted by -c N_e S in
  // the shifted FP32 mode: same eigenvectors, eigenvalue moved by -c N_e)
  for (size_t q = 0; q < pairs.size(); ++q) {
    const int i = pairs[q].first, j = pairs[q].second;
    const double h = er.H[q] + pb.e_core * er.S[q];
    out.H[i * M + j] = out.H[j * M + i] = h;
    out.S[i * M + j] = out.S[j * M + i] = er.S[q];
  }
  for (double v : out.H) require(std::isfinite(v), TNQE_ENONFINITE, "non-finite H element");
  for (double v : out.S) require(std::isfinite(v), TNQE_ENONFINITE, "non-finite S element");
  require(M <= kMaxM, TNQE_EINVAL, "M exceeds the device eigensolver limit");
  const double *dH = c.upload(out.H), *dS = c.upload(out.S);
  std::vector<int> Ms{M};
  std::vector<int64_t> offs{0};
  double *dout = c.dev<double>(8 + kMaxM);
  launch_gep(dH, dS, c.upload(Ms), c.upload(offs), 1, op.eps_S > 0 ? op.eps_S : 1e-12, dout, ctx->stream);
  c.check_launch();
  std::vector<double> go(8 + kMaxM);
  TNQE_HIP(hipMemcpyAsync(go.data(), dout, go.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  c.sync();
  rep.t_gep_ms = ms_since(tq);
  require(go[5] == 0.0, TNQE_ESINGULAR, "S has no eigenvalue above the threshold");
  out.E = go[0] + shift_total;
  out.c.assign(go.begin() + 8, go.begin() + 8 + M);
  rep.cond_S = go[1];
  rep.lambda_min_S = go[2];
  rep.n_dropped = (int)go[3];
  rep.kappa1 = go[4];
  if (shift_total != 0.0) {
    // back to H: H' + c N_e S; kappa_1 of the unshifted eigenvalue (App. A2)
    for (int x = 0; x < M * M; ++x) out.H[x] += shift_total * out.S[x];
    double cc = 0.0;
    for (double v : out.c) cc += v * v;
    rep.kappa1 = cc / std::sqrt(out.E * out.E + 1.0);
  }
  rep.max_discarded_weight_sum = 0.0;
  for (double d : ts.discarded) rep.max_discarded_weight_sum = std::max(rep.max_discarded_weight_sum, d);
  rep.min_rel_gap = ts.min_gap;
  rep.env_flops = er.flops;
  for (int k = 0; k < kEnvKinds; ++k) {
    rep.env_kind_ms[k] = er.kind_ms[k];
    rep.env_kind_flops[k] = er.kind_flops[k];
    rep.env_kind_bytes[k] = er.kind_bytes[k];
    rep.env_kind_launches[k] = er.kind_launches[k];
  }
  rep.alg_bytes = er.bytes;
  rep.env_kernel_ms = er.kernel_ms;
  rep.svd_kernel_ms = ts.svd.ms;
  rep.svd_flops = ts.svd.flops;
  rep.svd_launches = ts.svd.launches;
  rep.move_kernel_ms = ts.svd.cat_ms[kCatMove];
  rep.move_flops = ts.svd.cat_flops[kCatMove];
  rep.move_launches = ts.svd.cat_launches[kCatMove];
  rep.t_moves_ms = ts.move_wall_ms;
  rep.t_tune_ms = er.tune_ms;
  for (int k = 0; k < kFactKinds; ++k) {
    rep.svd_kind_ms[k] = ts.svd.kind_ms[k];
    rep.svd_kind_flops[k] = ts.svd.kind_flops[k];
    rep.svd_kind_launches[k] = ts.svd.kind_launches[k];
  }
  rep.alg_flops = er.flops + ts.svd.flops;
  rep.n_pairs = (int)pairs.size();
  rep.max_bond = std::max(ts.max_bond, er.max_pad);
  rep.mpo_max_bond = mpo.max_bond;
  rep.t_total_ms = ms_since(t0);
  require(std::isfinite(out.E), TNQE_ENONFINITE, "non-finite eigenvalue");
}


// ------------------------------------------------------------ expanded one-hot pencil
// Bond dimensions per sector of state i after the canonical form used for the
// expansion: left-canonicalised by exact QR (centre on the last site), then
// moved by exact LQ to site p (a block of R x C keeps min(R, C) vectors).
std::vector<std::vector<int>> onehot_dims(const tnqe_problem &pb, int i, int p) {
  const int N = pb.N, nb1 = pb.nb + 1, nslot = pb.nslot();
  std::vector<std::vector<int>> d = pb.mps[i].secdim;
  auto at = [&](int b, int a, int bb) { return (a < 0 || bb < 0 || a > pb.na || bb > pb.nb) ? 0 : d[b][a * nb1 + bb]; };
  for (int b = 1; b < N; ++b)
    for (int s = 0; s < nslot; ++s) {
      const int sa = s / nb1, sb = s % nb1;
      int R = 0;
      for (int k = 0; k < 4; ++k) R += at(b - 1, sa - qk_a(k), sb - qk_b(k));
      d[b][s] = std::min(R, d[b][s]);
    }
  for (int q = N - 1; q > p; --q)
    for (int s = 0; s < nslot; ++s) {
      const int sa = s / nb1, sb = s % nb1;
      int C = 0;
      for (int k = 0; k < 4; ++k) C += at(q + 1, sa + qk_a(k), sb + qk_b(k));
      d[q][s] = std::min(d[q][s], C);
    }
  return d;
}

// One-hot entries (l, k_p, k_{p+1}, r) of the two-site tensor at (p, p+1)
// that conserve the particle numbers, in row-major order of T.
std::vector<int4> onehot_list(const tnqe_problem &pb, const std::vector<std::vector<int>> &d, int p) {
  const int nb1 = pb.nb + 1, nslot = pb.nslot();
  std::vector<int> off0(nslot + 1, 0), off2(nslot + 1, 0);
  for (int s = 0; s < nslot; ++s) {
    off0[s + 1] = off0[s] + d[p][s];
    off2[s + 1] = off2[s] + d[p + 2][s];
  }
  std::vector<int4> out;
  for (int s = 0; s < nslot; ++s) {
    const int sa = s / nb1, sb = s % nb1;
    for (int l = off0[s]; l < off0[s + 1]; ++l)
      for (int kp = 0; kp < 4; ++kp)
        for (int kq = 0; kq < 4; ++kq) {
          const int a = sa + qk_a(kp) + qk_a(kq), b = sb + qk_b(kp) + qk_b(kq);
          if (a > pb.na || b > pb.nb) continue;
          const int s2 = a * nb1 + b;
          for (int r = off2[s2]; r < off2[s2 + 1]; ++r) out.push_back(make_int4(l, kp, kq, r));
        }
  }
  // sectors are contiguous in every bond, so sorting restores row-major order
  std::sort(out.begin(), out.end(), [](const int4 &x, const int4 &y) {
    return std::make_tuple(x.x, x.y, x.z, x.w) < std::make_tuple(y.x, y.y, y.z, y.w);
  });
  return out;
}

struct OneHotOut {
  std::vector<int4> index;
  std::vector<double> Hd, Sd, Hc, Sc;
};

// the pencil blocks on the device (valid while the Call lives), and state ei
// in the canonical form centred on p
struct OneHotDev {
  std::vector<int4> index;
  std::vector<int> dense_of;        // index m -> ((l * 4 + k_p) * 4 + k_{p+1}) * Dq + r
  const int *d_dense = nullptr;
  std::vector<int> dmap;            // dense index -> m (-1: not a one-hot entry)
  const int4 *d_oh = nullptr;       // the index on the device
  const int *d_map = nullptr;       // dmap on the device
  double *Hd = nullptr, *Sd = nullptr, *Hc = nullptr, *Sc = nullptr;   // [n][n], [n][n], [n][M], [n][M]
  KetSet ci;
  int Dp = 0, Dq = 0;               // total dimensions of bonds p and p + 2
};

// Expanded pencil of state ei at sites (p, p+1) (App. A1, single expanded
// state): ei in canonical form centred on p; for every state k the ket is k
// rotated into basis ei by its Givens network with truncation (k = ei: ei
// itself); left environments over sites < p and right environments over
// sites > p + 1 with the dense MPO of H^(ei) (and with the identity for the
// overlaps), then the two-site blocks.  Every contraction is a matrix-core
// GEMM (launch_oh_gemm).
void onehot_core(Call &c, tnqe_problem &pb, const tnqe_options &op, int ei, int p, OneHotDev &out,
                 tnqe_report &rep) {
  tnqe_ctx *ctx = c.ctx;
  const auto t0 = Clock::now();
  const int N = pb.N, M = pb.M;
  require(ei >= 0 && ei < M, TNQE_EINVAL, "expanded state out of range");
  require(p >= 0 && p + 1 < N, TNQE_EINVAL, "two-site position out of range");
  const int chi_cap = op.chi_cap_override > 0 ? op.chi_cap_override : op.chi;
  const int max_sweeps = op.max_sweeps > 0 ? op.max_sweeps : 40;
  rep = tnqe_report{};
  hipStream_t st = ctx->stream;
  // ---- dense MPO of H^(ei), site by site: W_x[w][w'][k'][k]
  MpoStructure &mpo = mpo_for(ctx, N);
  std::vector<double> hi, gi, vals, slotv;
  rotate_integrals(pb, pb.mps[ei].U, hi, gi);
  mpo_values(mpo, hi.data(), gi.data(), vals, slotv);
  std::vector<std::vector<int>> base(N + 1);
  std::vector<int> D(N + 1, 0);
  for (int b = 0; b <= N; ++b)
    for (const MpoClass &cl : mpo.classes[b]) {
      base[b].push_back(D[b]);
      D[b] += cl.nw;
    }
  std::vector<const double *> dW(N);
  for (int x = 0; x < N; ++x) {
    std::vector<double> Wx((size_t)D[x] * D[x + 1] * 16, 0.0);
    for (const MpoGroup &grp : mpo.groups[x]) {
      const OpPattern &P = mpo.patterns[grp.pattern];
      const double *gv = vals.data() + mpo.site_nnz_off[x] + grp.val_off;
      auto add = [&](int r, int col, double v) {
        const int64_t wi = base[x][grp.cin] + col, wo = base[x + 1][grp.cout] + r;
        for (int e = 0; e < P.n; ++e) Wx[((wi * D[x + 1] + wo) * 4 + P.kp[e]) * 4 + P.k[e]] += v * P.f[e];
      };
      if (grp.dense) {
        for (int r = 0; r < grp.nr; ++r)
          for (int cc = 0; cc < grp.nc; ++cc) add(grp.r0 + r, grp.c0 + cc, gv[(int64_t)r * grp.nc + cc]);
      } else {
        for (int r = 0; r + 1 < (int)grp.rowptr.size(); ++r)
          for (int z = grp.rowptr[r]; z < grp.rowptr[r + 1]; ++z) add(r, grp.col[z], gv[z]);
      }
    }
    dW[x] = c.upload(Wx);
  }
  std::vector<double> Wid(16, 0.0);
  for (int k = 0; k < 4; ++k) Wid[k * 4 + k] = 1.0;
  const double *dWid = c.upload(Wid);
  const int wH = base[N][mpo.final_class] + mpo.final_H;
  const int wIp = base[p][mpo.I_class[p]] + mpo.I_loc[p];
  // ---- every other state rotated into basis ei; ei centred on p
  const auto tg = Clock::now();
  std::vector<std::pair<int, int>> offd;
  for (int k = 0; k < M; ++k)
    if (k != ei) offd.push_back({ei, k});
  const int P = (int)offd.size();
  KetSet canon, kets;
  TruncStats ts;
  gate_phase(c, pb, offd, chi_cap, op, max_sweeps, canon, kets, ts);
  const std::vector<int> cap = bond_caps(pb, chi_cap);
  KetSet &ci = out.ci;
  ci.init(&c, 1, N, pb.na, pb.nb, cap);
  {
    std::vector<double *> dst(1), src(1);
    std::vector<int64_t> cnt(1);
    for (int x = 0; x < N; ++x) {
      dst[0] = ci.site_ptr[x];
      src[0] = canon.site_ptr[(size_t)ei * N + x];
      cnt[0] = (int64_t)canon.htot[(size_t)x * M + ei] * 4 * canon.htot[(size_t)(x + 1) * M + ei];
      launch_copy(c.upload(dst), c.upload(src), c.upload(cnt), 1, st);
    }
    for (int b = 0; b <= N; ++b) {
      for (int s2 = 0; s2 < pb.nslot(); ++s2) ci.dim(b, 0, s2) = canon.dim(b, ei, s2);
      ci.commit_bond(b);
    }
    for (int q = N - 1; q > p; --q) {
      const size_t mm = ctx->pool.mark();
      move_left(ci, q, max_sweeps, &ts.svd);
      ctx->pool.rewind(mm);
    }
    c.sync();
  }
  // the dense contractions below read whole site tensors: clear what lies
  // outside the quantum-number blocks
  for (int x = 0; x < N; ++x) {
    int64_t mx = 0;
    for (int t = 0; t < P; ++t) mx = std::max<int64_t>(mx, (int64_t)kets.htot[(size_t)x * P + t] * 4 * kets.htot[(size_t)(x + 1) * P + t]);
    if (P > 0) launch_mask_site(kets.tables(), x, (int)std::min<int64_t>(mx, INT32_MAX), st);
    launch_mask_site(ci.tables(), x, ci.htot[x] * 4 * ci.htot[x + 1], st);
  }
  c.check_launch();
  c.sync();
  ts.svd.collect(ctx);
  rep.t_gates_ms = ms_since(tg);
  // ---- one-hot entries (the host planned the same dimensions the moves produced)
  {
    const std::vector<std::vector<int>> dchk = onehot_dims(pb, ei, p);
    for (int b : {p, p + 2})
      for (int s2 = 0; s2 < pb.nslot(); ++s2)
        require(dchk[b][s2] == ci.dim(b, 0, s2), TNQE_ESHAPE, "canonical bond dimensions differ from the plan");
  }
  std::vector<std::vector<int>> dci(N + 1, std::vector<int>(pb.nslot()));
  for (int b = 0; b <= N; ++b)
    for (int s2 = 0; s2 < pb.nslot(); ++s2) dci[b][s2] = ci.dim(b, 0, s2);
  out.index = onehot_list(pb, dci, p);
  const int n = (int)out.index.size();
  require(n > 0, TNQE_ESHAPE, "the two-site tensor has no entries in the particle-number sector");
  const int Dbp = ci.htot[p], Dbm = ci.htot[p + 1], Dbq = ci.htot[p + 2];
  std::vector<int> &dense_of = out.dense_of, &dmap = out.dmap;
  dmap.assign((size_t)Dbp * 16 * Dbq, -1);
  dense_of.resize(n);
  out.Dp = Dbp;
  out.Dq = Dbq;
  for (int m = 0; m < n; ++m) {
    const int4 &e = out.index[m];
    dense_of[m] = ((e.x * 4 + e.y) * 4 + e.z) * Dbq + e.w;
    dmap[dense_of[m]] = m;
  }
  const int *d_dense = c.upload(dense_of);
  out.d_dense = d_dense;
  const int *d_map = c.upload(dmap);
  const int4 *d_oh = c.upload(out.index);
  out.d_map = d_map;
  out.d_oh = d_oh;
  double *dHc = c.dev<double>((size_t)n * M), *dSc = c.dev<double>((size_t)n * M);
  double *dHd = c.dev<double>((size_t)n * n), *dSd = c.dev<double>((size_t)n * n);
  out.Hc = dHc;
  out.Sc = dSc;
  out.Hd = dHd;
  out.Sd = dSd;
  (void)Dbm;
  // ---- environments and blocks, pair by pair
  const auto te = Clock::now();
  double flops = 0.0;
  auto gemm = [&](int kind, int Mm, int Nn, int Kk, const double *A, const double *B, double *C, int d0 = 0,
                  int d1 = 0, int d2 = 0, const int *map = nullptr) {
    OhGemm g{};
    g.kind = kind;
    g.M = Mm;
    g.N = Nn;
    g.K = Kk;
    g.A = A;
    g.B = B;
    g.C = C;
    g.d0 = d0;
    g.d1 = d1;
    g.d2 = d2;
    g.map = map;
    g.n_oh = n;
    launch_oh_gemm(g, st);
    flops += 2.0 * Mm * Nn * Kk;
  };
  TNQE_HIP(hipEventRecord(ctx->ev[2], st));
  for (int k = 0; k < M; ++k) {
    const size_t mk = ctx->pool.mark();
    const int t = k < ei ? k : k - 1;
    auto ket = [&](int x) -> const double * { return k == ei ? ci.site_ptr[x] : kets.site_ptr[(size_t)t * N + x]; };
    auto Dk = [&](int b) { return k == ei ? ci.htot[b] : kets.htot[(size_t)b * P + t]; };
    auto Db = [&](int b) { return ci.htot[b]; };
    // buffer sizes over the sweep
    int64_t envmax = 1, xmax = 1;
    for (int x = 0; x < N; ++x) {
      envmax = std::max(envmax, (int64_t)D[x] * Db(x) * Dk(x));
      xmax = std::max(xmax, (int64_t)std::max(D[x], D[x + 1]) * 4 * std::max(Db(x), Db(x + 1)) *
                                std::max(Dk(x), Dk(x + 1)));
    }
    envmax = std::max(envmax, (int64_t)D[N]);
    double *E0 = c.dev<double>(envmax), *E1 = c.dev<double>(envmax);
    double *X = c.dev<double>(xmax), *Y = c.dev<double>(xmax);
    // left environment at bond p
    {
      std::vector<double> L0(D[0], 0.0);
      L0[base[0][mpo.I_class[0]] + mpo.I_loc[0]] = 1.0;
      c.upload_to(E0, L0.data(), L0.size());
    }
    double *Lc = E0, *Ln = E1;
    for (int x = 0; x < p; ++x) {
      gemm(kOhPlain, D[x] * Db(x), 4 * Dk(x + 1), Dk(x), Lc, ket(x), X);
      gemm(kOhWX, D[x + 1] * 4, Db(x) * Dk(x + 1), D[x] * 4, dW[x], X, Y, D[x + 1], Db(x), Dk(x + 1));
      gemm(kOhBraL, Db(x + 1), D[x + 1] * Dk(x + 1), 4 * Db(x), ci.site_ptr[x], Y, Ln, Db(x), Dk(x + 1));
      std::swap(Lc, Ln);
    }
    double *Lp = c.dev<double>((size_t)D[p] * Db(p) * Dk(p));
    TNQE_HIP(hipMemcpyAsync(Lp, Lc, sizeof(double) * D[p] * Db(p) * Dk(p), hipMemcpyDeviceToDevice, st));
    // right environments at bond p + 2: H (boundary: the final H channel) and
    // the overlap (identity operator)
    double *Rq[2] = {c.dev<double>((size_t)D[p + 2] * Db(p + 2) * Dk(p + 2)),
                     c.dev<double>((size_t)Db(p + 2) * Dk(p + 2))};
    for (int which = 0; which < 2; ++which) {
      auto Dw = [&](int b) { return which == 0 ? D[b] : 1; };
      std::vector<double> RN(Dw(N), 0.0);
      RN[which == 0 ? wH : 0] = 1.0;
      c.upload_to(E0, RN.data(), RN.size());
      double *Rc = E0, *Rn = E1;
      for (int x = N - 1; x >= p + 2; --x) {
        const double *Wx = which == 0 ? dW[x] : dWid;
        gemm(kOhPlainBT, Dw(x + 1) * Db(x + 1), Dk(x) * 4, Dk(x + 1), Rc, ket(x), X);
        gemm(kOhRX2, Dw(x) * 4, Db(x + 1) * Dk(x), Dw(x + 1) * 4, Wx, X, Y, Dw(x + 1));
        gemm(kOhBraR, Db(x), Dw(x) * Dk(x), 4 * Db(x + 1), ci.site_ptr[x], Y, Rn, Dk(x));
        std::swap(Rc, Rn);
      }
      TNQE_HIP(hipMemcpyAsync(Rq[which], Rc, sizeof(double) * Dw(p + 2) * Db(p + 2) * Dk(p + 2),
                              hipMemcpyDeviceToDevice, st));
    }
    const double *LS = Lp + (int64_t)wIp * Db(p) * Dk(p);
    // column k: <varphi_m|H|ket> and <varphi_m|ket>
    const int b0 = Db(p), k0 = Dk(p), k2 = Dk(p + 2), b2 = Db(p + 2);
    double *Th = c.dev<double>((size_t)4 * k0 * 4 * k2);
    double *t1 = c.dev<double>((size_t)D[p] * b0 * 16 * k2);
    double *t2 = c.dev<double>((size_t)D[p + 1] * 4 * b0 * 4 * k2);
    double *t3 = c.dev<double>((size_t)D[p + 2] * 4 * 4 * b0 * k2);
    double *VH = c.dev<double>((size_t)b0 * 16 * b2), *VS = c.dev<double>((size_t)b0 * 16 * b2);
    double *s1 = c.dev<double>((size_t)b0 * 16 * k2);
    gemm(kOhPlain, 4 * k0, 4 * k2, Dk(p + 1), ket(p), ket(p + 1), Th);
    gemm(kOhPlain, D[p] * b0, 16 * k2, k0, Lp, Th, t1);
    gemm(kOhWX, D[p + 1] * 4, b0 * 4 * k2, D[p] * 4, dW[p], t1, t2, D[p + 1], b0, 4 * k2);
    gemm(kOhA3, D[p + 2] * 4, 4 * b0 * k2, D[p + 1] * 4, dW[p + 1], t2, t3, D[p + 2], b0, k2);
    gemm(kOhA4, b0 * 16, b2, D[p + 2] * k2, t3, Rq[0], VH, b0, k2, b2);
    gemm(kOhPlain, b0, 16 * k2, k0, LS, Th, s1);
    gemm(kOhPlainBT, 16 * b0, b2, k2, s1, Rq[1], VS);
    launch_oh_gather(VH, VS, pb.e_core, d_dense, n, dHc, M, k, st);
    launch_oh_gather(VS, nullptr, 0.0, d_dense, n, dSc, M, k, st);
    if (k == ei) {
      // diagonal block: L (x) W_p W_{p+1} (x) R over every pair of one-hot entries
      double *Z1 = c.dev<double>((size_t)D[p] * 16 * D[p + 2] * 16);
      double *Z2 = c.dev<double>((size_t)b0 * b0 * 256 * D[p + 2]);
      gemm(kOhD1, D[p] * 16, D[p + 2] * 16, D[p + 1], dW[p], dW[p + 1], Z1, D[p + 1]);
      gemm(kOhPlainAT, b0 * b0, 256 * D[p + 2], D[p], Lp, Z1, Z2);
      gemm(kOhD3, b0 * b0 * 256, b2 * b2, D[p + 2], Z2, Rq[0], dHd, b0, D[p + 2], b2, d_map);
      launch_oh_sd(d_oh, n, LS, b0, Rq[1], b2, pb.e_core, dSd, dHd, st);
    }
    c.check_launch();
    c.sync();
    ctx->pool.rewind(mk);
  }
  TNQE_HIP(hipEventRecord(ctx->ev[3], st));
  c.sync();
  float ms = 0.0f;
  TNQE_HIP(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
  rep.t_env_ms = ms_since(te);
  rep.env_kernel_ms = ms;
  rep.env_flops = flops;
  rep.svd_kernel_ms = ts.svd.ms;
  rep.svd_flops = ts.svd.flops;
  rep.alg_flops = flops + ts.svd.flops;
  rep.max_discarded_weight_sum = 0.0;
  for (double dd : ts.discarded) rep.max_discarded_weight_sum = std::max(rep.max_discarded_weight_sum, dd);
  rep.min_rel_gap = ts.min_gap;
  rep.n_pairs = M;
  rep.mpo_max_bond = mpo.max_bond;
  rep.t_total_ms = ms_since(t0);
}

void onehot_one(tnqe_ctx *ctx, tnqe_problem &pb, const tnqe_options &op, int ei, int p, OneHotOut &out,
                tnqe_report &rep) {
  Call c{ctx};
  OneHotDev dv;
  onehot_core(c, pb, op, ei, p, dv, rep);
  const size_t n = dv.index.size(), M = pb.M;
  out.index = dv.index;
  out.Hd.resize(n * n);
  out.Sd.resize(n * n);
  out.Hc.resize(n * M);
  out.Sc.resize(n * M);
  hipStream_t st = ctx->stream;
  TNQE_HIP(hipMemcpyAsync(out.Hd.data(), dv.Hd, out.Hd.size() * 8, hipMemcpyDeviceToHost, st));
  TNQE_HIP(hipMemcpyAsync(out.Sd.data(), dv.Sd, out.Sd.size() * 8, hipMemcpyDeviceToHost, st));
  TNQE_HIP(hipMemcpyAsync(out.Hc.data(), dv.Hc, out.Hc.size() * 8, hipMemcpyDeviceToHost, st));
  TNQE_HIP(hipMemcpyAsync(out.Sc.data(), dv.Sc, out.Sc.size() * 8, hipMemcpyDeviceToHost, st));
  c.sync();
  for (double v : out.Hd) require(std::isfinite(v), TNQE_ENONFINITE, "non-finite one-hot element");
  for (double v : out.Hc) require(std::isfinite(v), TNQE_ENONFINITE, "non-finite one-hot element");
}

// ------------------------------------------------------------ generalized-sweep step
// One step of Alg. A.1 at sites (p, p+1) for the expanded state ei (App. A1:
// one chosen reference state; no single-site mitigation repetitions): the
// expanded pencil in the order of eq. subs_exp, the discard of dependent
// columns (App. A2), the thresholded eigenproblem (eq. exp_gen_eig), the
// parameter update (eq. param_upd), the rotation of the bond (App. A3), the
// truncation to chi and the merge of the rotation into the orbital basis.
struct SweepOut {
  double E_old = 0.0, E1 = 0.0, E_new = 0.0, theta = 0.0, xi_none = 0.0, xi = 0.0, discarded = 0.0;
  int n = 0, D = 0, n_kept = 0, n_dropped_S = 0, accepted = 0, new_bond = 0, mit_columns = 0, mit_kept = 0;
  std::vector<double> tnew;
  std::vector<int32_t> bond_dim;
  std::vector<int32_t> bond_qn;
  std::vector<double> sites, U;
};

// FSWAP f4 on (k_p, k_{p+1}) (App. A3): (1 x f2 x 1)(f2 x f2)(1 x f2 x 1) in
// the mode basis (p up, p down, p+1 up, p+1 down), entry x = row * 16 + col
double fswap4_entry(int x) {
  static const int kq[4] = {0, 2, 1, 3};   // local state k -> mode bits (n_up, n_dn)
  static const double f2[16] = {1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, -1};
  const int I = kq[x >> 6] * 4 + kq[(x >> 4) & 3], J = kq[(x >> 2) & 3] * 4 + kq[x & 3];
  // (1 x f2 x 1) maps mode bits 1, 2 of a row through f2 (a permutation with a sign)
  static const int f2c[4] = {0, 2, 1, 3};
  static const double f2s[4] = {1.0, 1.0, 1.0, -1.0};
  const int ci = (I & 8) | (f2c[(I >> 1) & 3] << 1) | (I & 1), cj = (J & 8) | (f2c[(J >> 1) & 3] << 1) | (J & 1);
  const double si = f2s[(I >> 1) & 3], sj = f2s[(J >> 1) & 3];
  return si * f2[(ci >> 2) * 4 + (cj >> 2)] * f2[(ci & 3) * 4 + (cj & 3)] * sj + 0.0;
}

// a rotation is taken only when it lowers xi by more than this: xi is a
// difference of order-one sums, and below it the choice would be rounding
constexpr double kXiTol = 1e-12;

using Gate16 = std::array<double, 256>;
Gate16 givens_gate(double theta) {
  Gate16 g;
  const double c = std::cos(theta), s = std::sin(theta);
  for (int x = 0; x < 256; ++x) g[x] = gate4_entry(c, s, x);
  return g;
}
Gate16 fswap_gate() {
  Gate16 g;
  for (int x = 0; x < 256; ++x) g[x] = fswap4_entry(x);
  return g;
}

// Quantum-number blocks of the two-site matrix (l, k_p) x (k_{p+1}, r) of
// state ci at (p, p+1) for every gate of a list, with their SVDs done:
// blocks of gate g are first[g] .. first[g+1] (pair = g), in sector order.
struct RotatedBlocks {
  std::vector<Blk> blks;
  std::vector<int> first;
  Blk *dblk = nullptr;
  double *scratch = nullptr;
  int max_values = 0;
};
void rotated_blocks(Call &c, KetSet &ci, int p, const double *dT, const std::vector<Gate16> &gates, int max_sweeps,
                    RotatedBlocks &rb) {
  const int nslot = ci.nslot, nb1 = ci.nb + 1;
  std::vector<int> offp(nslot), offq(nslot);
  for (int s = 0; s < nslot; ++s) {
    offp[s] = ci.hbtab[((size_t)p * ci.n) * nslot + s].x;
    offq[s] = ci.hbtab[((size_t)(p + 2) * ci.n) * nslot + s].x;
  }
  std::vector<Blk> one;
  for (int s = 0; s < nslot; ++s) {
    const int sa = s / nb1, sb = s % nb1;
    Blk b{};
    b.sa = sa;
    b.sb = sb;
    b.rs[0] = b.cs[0] = 0;
    for (int k = 0; k < 4; ++k) {
      b.rs[k + 1] = b.rs[k] + ci.dim_q(p, 0, sa - qk_a(k), sb - qk_b(k));
      b.cs[k + 1] = b.cs[k] + ci.dim_q(p + 2, 0, sa + qk_a(k), sb + qk_b(k));
    }
    b.R = b.rs[4];
    b.C = b.cs[4];
    if (b.R == 0 || b.C == 0) continue;
    plan_block(b);
    one.push_back(b);
  }
  Scratch sc;
  rb.blks.clear();
  rb.first.assign(1, 0);
  rb.max_values = 0;
  for (size_t g = 0; g < gates.size(); ++g) {
    int nv = 0;
    for (Blk b : one) {
      b.pair = (int)g;
      take_block_storage(b, sc);
      b.offS = sc.take(b.n);
      b.kept = b.n;
      nv += b.n;
      rb.blks.push_back(b);
    }
    rb.first.push_back((int)rb.blks.size());
    rb.max_values = std::max(rb.max_values, nv);
  }
  require(rb.max_values <= kXiMaxValues, TNQE_ESHAPE, "two-site matrix with too many singular values");
  rb.scratch = c.dev<double>(sc.used);
  std::vector<double> gflat(gates.size() * 256);
  for (size_t g = 0; g < gates.size(); ++g) std::copy(gates[g].begin(), gates[g].end(), gflat.begin() + g * 256);
  Call::Blob bl;
  const size_t o_blk = bl.add(rb.blks), o_g = bl.add(gflat), o_p = bl.add(offp), o_q = bl.add(offq);
  char *base = c.upload(bl);
  rb.dblk = Call::at<Blk>(base, o_blk);
  launch_sw_gate_blocks(rb.dblk, (int)rb.blks.size(), Call::at<const double>(base, o_g), dT, ci.htot[p + 2],
                        Call::at<const int>(base, o_p), Call::at<const int>(base, o_q), ci.na, nb1, rb.scratch,
                        c.ctx->stream);
  run_svd(c, rb.dblk, rb.blks, max_sweeps, rb.scratch);
  c.check_launch();
}

// xi (App. A3) of every gate of the list
std::vector<double> truncation_errors(Call &c, KetSet &ci, int p, const double *dT, const std::vector<Gate16> &gates,
                                      int chi, int max_sweeps) {
  const size_t mk = c.ctx->pool.mark();
  RotatedBlocks rb;
  rotated_blocks(c, ci, p, dT, gates, max_sweeps, rb);
  double *dxi = c.dev<double>(gates.size());
  launch_sw_xi(rb.dblk, c.upload(rb.first), (int)gates.size(), rb.max_values, rb.scratch, chi, dxi, c.ctx->stream);
  c.check_launch();
  std::vector<double> xi(gates.size());
  TNQE_HIP(hipMemcpyAsync(xi.data(), dxi, xi.size() * sizeof(double), hipMemcpyDeviceToHost, c.ctx->stream));
  c.sync();
  c.ctx->pool.rewind(mk);
  return xi;
}

// eigen- (singular) decomposition of a symmetric positive semi-definite n x n
// device matrix by the Jacobi SVD: vectors by row ([n][n]) and values, both
// in decreasing order of the values.  Matrices too wide for the register
// kernels take the global-memory Jacobi with its sweeps spread over the chip
// by blocks of columns (path 0).  At any n, path 1 forces the one-workgroup
// global-memory kernel, path 2 the chip-wide one by column pairs (the same
// bits as path 1) and path 3 the chip-wide one by column blocks.
// the two instantiated sweep graphs of a chip-wide eigensolve (one per
// control slot), released when the solve returns or throws (after the stream
// they were launched on has drained)
struct SweepGraphs {
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipStream_t stream = nullptr;
  explicit SweepGraphs(hipStream_t st) : stream(st) {}
  SweepGraphs(const SweepGraphs &) = delete;
  SweepGraphs &operator=(const SweepGraphs &) = delete;
  ~SweepGraphs() {
    if (exec[0] || exec[1]) (void)hipStreamSynchronize(stream);
    for (hipGraphExec_t e : exec)
      if (e) (void)hipGraphExecDestroy(e);
  }
};

void psd_eigen(Call &c, const double *A, int n, int max_sweeps, double *&vec, double *&val, int path = 0) {
  Blk b{};
  b.R = b.C = n;
  b.rs[0] = b.cs[0] = 0;
  for (int k = 1; k <= 4; ++k) b.rs[k] = b.cs[k] = n;
  plan_block(b);
  if (path != 0) b.offW = 0;   // global-memory storage
  const bool wide = b.offW >= 0 && path != 1;
  const bool blocked = path == 0 || path == 3 || path == 4;
  const bool graphs = path == 0 || path == 3;
  Scratch sc;
  take_block_storage(b, sc);
  b.offS = sc.take(n);
  b.kept = n;
  double *scratch = c.dev<double>(sc.used);
  hipStream_t st = c.ctx->stream;
  TNQE_HIP(hipMemcpyAsync(scratch + b.offT, A, sizeof(double) * n * n, hipMemcpyDeviceToDevice, st));
  std::vector<Blk> blks{b};
  Blk *dblk = c.upload(blks);
  if (!wide) {
    run_svd(c, dblk, blks, max_sweeps, scratch);
  } else {
    // the sweep loop on the host: one sync per sweep to read its rotation flag
    const int *didx = c.upload(std::vector<int>{0});
    unsigned long long *ctl = c.dev<unsigned long long>(4);
    launch_jacobi_wide_load(dblk, didx, scratch, ctl, st);
    // a blocked sweep is 1 + (blocks - 1) launches with the same arguments in
    // every sweep of the same control slot: each slot's sequence is captured
    // once into a graph and replayed on the call's stream (kernel nodes only;
    // captured on a side stream of the library, since the caller's stream
    // may be the null stream, which cannot be captured)
    SweepGraphs sg(st);
    hipStream_t cst = c.ctx->aux[0];
    if (graphs) prepare_jacobi_wide_sweep_blocked();
    int sweep = 0;
    for (; sweep < max_sweeps && n > 1; ++sweep) {
      const int slot = sweep & 1;
      if (graphs) {
        if (!sg.exec[slot]) {
          TNQE_HIP(hipStreamBeginCapture(cst, hipStreamCaptureModeRelaxed));
          hipGraph_t g = nullptr;
          try {
            launch_jacobi_wide_sweep_blocked(scratch + b.offW, n, n, ctl, slot, cst);
          } catch (...) {
            (void)hipStreamEndCapture(cst, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
          }
          TNQE_HIP(hipStreamEndCapture(cst, &g));
          const hipError_t e = hipGraphInstantiate(&sg.exec[slot], g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          TNQE_HIP(e);
        }
        TNQE_HIP(hipGraphLaunch(sg.exec[slot], st));
      } else if (blocked) {
        launch_jacobi_wide_sweep_blocked(scratch + b.offW, n, n, ctl, slot, st);
      } else {
        launch_jacobi_wide_sweep(scratch + b.offW, n, n, ctl, slot, st);
      }
      unsigned long long rot = 0;
      TNQE_HIP(hipMemcpyAsync(&rot, ctl + 2 + slot, sizeof(rot), hipMemcpyDeviceToHost, st));
      c.sync();
      if ((rot & 2) == 0) break;   // no rotation of a pair not yet orthogonal to 1e-10
    }
    launch_jacobi_wide_finish(dblk, didx, scratch, sweep, nullptr, st);
  }
  c.check_launch();
  vec = scratch + b.offU;
  val = scratch + b.offS;
}

void sw_gemm(Call &c, int kind, int Mm, int Nn, int Kk, const double *A, const double *B, double *C) {
  OhGemm g{};
  g.kind = kind;
  g.M = Mm;
  g.N = Nn;
  g.K = Kk;
  g.A = A;
  g.B = B;
  g.C = C;
  launch_oh_gemm(g, c.ctx->stream);
}

// Steps 2-4 on an expanded pencil whose state-ei block is spanned by n
// orthonormal states (device Hd, Sd [n][n], Hc, Sc [n][M]): the combined
// order of eq. subs_exp, the discard of dependent columns, the
// projection-thresholded lowest root, and the normalised coefficients of the
// n states (tnew, device [n]) signed against told (device, stride told_ld);
// with dense_of and T non-null they are scattered into the dense tensor T.
struct ExpandedRoot {
  double E = 0.0;
  int D = 0, n_kept = 0, n_dropped_S = 0;
};
ExpandedRoot expanded_root(Call &c, const double *dH, const double *dS, int M, int ei, int n, const double *Hd,
                           const double *Sd, const double *Hc, const double *Sc, const double *told, int told_ld,
                           double tol_ld, double eps_S, int max_sweeps, double *tnew, const int *dense_of, double *T,
                           int64_t tsize) {
  hipStream_t st = c.ctx->stream;
  ExpandedRoot er;
  const int D = n + M - 1;
  er.D = D;
  require(D <= 1024, TNQE_ESHAPE, "expanded pencil wider than 1024 columns");
  // combined order of eq. subs_exp and assembly
  std::vector<int> code(D);
  for (int a = 0; a < D; ++a) code[a] = a < ei ? -(a + 1) : a < ei + n ? a - ei : -(a - n + 1 + 1);
  double *Hx = c.dev<double>((size_t)D * D), *Sx = c.dev<double>((size_t)D * D);
  launch_sw_assemble(c.upload(code), D, n, M, dH, dS, Hd, Sd, Hc, Sc, Hx, Sx, st);
  // discard of linearly dependent columns
  double *A = c.dev<double>((size_t)D * D);
  int *dkeep = c.dev<int>(D);
  TNQE_HIP(hipMemcpyAsync(A, Sx, sizeof(double) * D * D, hipMemcpyDeviceToDevice, st));
  launch_sw_discard(A, Sx, D, tol_ld, dkeep, st);
  std::vector<int> keep(D);
  TNQE_HIP(hipMemcpyAsync(keep.data(), dkeep, D * sizeof(int), hipMemcpyDeviceToHost, st));
  c.sync();
  std::vector<int> kidx, col_of(D, -1);
  for (int a = 0; a < D; ++a)
    if (keep[a]) {
      col_of[a] = (int)kidx.size();
      kidx.push_back(a);
    }
  const int Dk = (int)kidx.size();
  er.n_kept = Dk;
  require(Dk >= 1, TNQE_ESINGULAR, "every column of the expanded pencil was discarded");
  double *Hk = c.dev<double>((size_t)Dk * Dk), *Sk = c.dev<double>((size_t)Dk * Dk);
  launch_sw_gather(Hx, Sx, D, c.upload(kidx), Dk, Hk, Sk, st);
  // projection-thresholded eigenproblem of the kept columns
  double *Uv = nullptr, *lam = nullptr;
  psd_eigen(c, Sk, Dk, max_sweeps, Uv, lam);
  std::vector<double> hl(Dk);
  TNQE_HIP(hipMemcpyAsync(hl.data(), lam, Dk * sizeof(double), hipMemcpyDeviceToHost, st));
  c.sync();
  int r = 0;
  while (r < Dk && hl[r] > eps_S * hl[0]) ++r;
  er.n_dropped_S = Dk - r;
  require(r >= 1, TNQE_ESINGULAR, "no overlap eigenvalue above the threshold");
  double *X = c.dev<double>((size_t)Dk * r), *Y = c.dev<double>((size_t)Dk * r), *Cm = c.dev<double>((size_t)r * r);
  double *Bm = c.dev<double>((size_t)r * r), *dshift = c.dev<double>(1), *ck = c.dev<double>(Dk);
  launch_sw_whiten(Uv, lam, Dk, r, X, st);
  sw_gemm(c, kOhPlain, Dk, r, Dk, Hk, X, Y);       // H_k X
  sw_gemm(c, kOhPlainAT, r, r, Dk, X, Y, Cm);      // X^T H_k X
  launch_sw_shift(Cm, r, Bm, dshift, st);
  double *Ub = nullptr, *sb = nullptr;
  psd_eigen(c, Bm, r, max_sweeps, Ub, sb);
  sw_gemm(c, kOhPlain, Dk, 1, r, X, Ub, ck);       // c' = X y (y: the first vector)
  double hs[2];
  TNQE_HIP(hipMemcpyAsync(&hs[0], dshift, sizeof(double), hipMemcpyDeviceToHost, st));
  TNQE_HIP(hipMemcpyAsync(&hs[1], sb, sizeof(double), hipMemcpyDeviceToHost, st));
  c.sync();
  er.E = hs[0] - hs[1];
  // parameter update (eq. param_upd)
  std::vector<int> col(n);
  for (int m = 0; m < n; ++m) col[m] = col_of[ei + m];
  double *dstat = c.dev<double>(2);
  launch_sw_update(ck, c.upload(col), told, told_ld, n, dense_of, T, tsize, tnew, dstat, st);
  c.check_launch();
  return er;
}

// Single-site mitigation (App. A4) after the truncation of a sweep step.  The
// expanded pencil is moved to the rotated basis (the gate in the one-hot
// basis, G: H^[ii] -> G^T H^[ii] G, H^[ik] -> G^T H^[ik]); then, nreps
// times, the state's two-site tensor X is expanded over single-site one-hot
// states at p and at p+1 with the other site held fixed: at p the fixed site
// is the orthonormal row basis V of X (its right singular vectors per
// sector), at p+1 the orthonormal column basis Q (its left singular vectors),
// with as many vectors per sector as the truncated bond holds.  A one-hot
// state of the expanded site times the fixed one is a combination of
// two-site one-hot states: rows of an isometry T, and the pencil block
// becomes T H T^T (and T H^[ik]).  Any orthonormal basis of the fixed site's
// space gives the same roots and updated X; the singular vectors are used
// here.  Returns the last root; A_p (= Q) and A_{p+1} (the updated site) on
// the host, centre at p+1.
struct MitOut {
  double E = 0.0;
  int columns = 0, kept = 0;
};
MitOut mitigate(Call &c, KetSet &ci, int p, const OneHotDev &dv, const Gate16 &G16, const double *dH,
                const double *dS, int M, int ei, const std::vector<int> &kept, int nreps, double tol_ld, double eps_S,
                int max_sweeps, std::vector<double> &Ap, std::vector<double> &Aq, int Dn) {
  hipStream_t st = c.ctx->stream;
  const int n = (int)dv.index.size(), Dp = dv.Dp, Dq = dv.Dq, nb1 = ci.nb + 1;
  const int64_t tsize = (int64_t)Dp * 16 * Dq;
  // the pencil in the rotated basis
  std::vector<double> g(G16.begin(), G16.end());
  double *Gm = c.dev<double>((size_t)n * n), *tmp = c.dev<double>((size_t)n * std::max(n, M));
  double *Hd2 = c.dev<double>((size_t)n * n), *Sd2 = c.dev<double>((size_t)n * n);
  double *Hc2 = c.dev<double>((size_t)n * M), *Sc2 = c.dev<double>((size_t)n * M);
  launch_sw_onehot_gate(dv.d_oh, dv.d_map, n, Dq, c.upload(g), Gm, st);
  sw_gemm(c, kOhPlain, n, n, n, dv.Hd, Gm, tmp);
  sw_gemm(c, kOhPlainAT, n, n, n, Gm, tmp, Hd2);
  sw_gemm(c, kOhPlain, n, n, n, dv.Sd, Gm, tmp);
  sw_gemm(c, kOhPlainAT, n, n, n, Gm, tmp, Sd2);
  sw_gemm(c, kOhPlainAT, n, M, n, Gm, dv.Hc, Hc2);
  sw_gemm(c, kOhPlainAT, n, M, n, Gm, dv.Sc, Sc2);
  // the truncated state's coefficients in the one-hot basis
  double *x = c.dev<double>(n), *dX = c.dev<double>(tsize);
  launch_sw_product(c.upload(Ap), c.upload(Aq), Dn, Dq, dv.d_oh, n, x, st);
  c.check_launch();
  auto offp = [&](int a, int b) { return ci.off_q(p, 0, a, b); };
  auto offq = [&](int a, int b) { return ci.off_q(p + 2, 0, a, b); };
  // sector of every index of bonds p, p+1 (new), p+2
  std::vector<int> secp(Dp), secq(Dq);
  for (int s = 0; s < ci.nslot; ++s) {
    for (int d = 0; d < ci.dim(p, 0, s); ++d) secp[ci.off_q(p, 0, s / nb1, s % nb1) + d] = s;
    for (int d = 0; d < ci.dim(p + 2, 0, s); ++d) secq[ci.off_q(p + 2, 0, s / nb1, s % nb1) + d] = s;
  }
  MitOut mo;
  const Gate16 ident = givens_gate(0.0);
  for (int rep = 0; rep < nreps; ++rep) {
    for (int site = p; site <= p + 1; ++site) {
      const size_t mk = c.ctx->pool.mark();
      launch_sw_scatter(x, n, dv.d_dense, dX, tsize, st);
      RotatedBlocks rb;
      rotated_blocks(c, ci, p, dX, {ident}, max_sweeps, rb);
      require(rb.blks.size() == kept.size(), TNQE_ESHAPE, "two-site blocks changed during the mitigation");
      std::vector<int> j0(kept.size() + 1, 0), blk_of_slot(ci.nslot, -1);
      for (size_t q = 0; q < kept.size(); ++q) {
        rb.blks[q].kept = kept[q];
        j0[q + 1] = j0[q] + kept[q];
        blk_of_slot[rb.blks[q].sa * nb1 + rb.blks[q].sb] = (int)q;
      }
      {
        Blk *dblk = c.upload(rb.blks);
        const std::vector<int> uf = unit_prefix(rb.blks, [](const Blk &b) { return factor_units(b); });
        launch_svd_factor(dblk, Units{c.upload(uf), (int)rb.blks.size(), uf.back()}, rb.scratch, st);
        c.check_launch();
      }
      std::vector<std::vector<double>> U(kept.size()), B(kept.size()), sv(kept.size());
      for (size_t q = 0; q < kept.size(); ++q) {
        const Blk &b = rb.blks[q];
        U[q].resize((size_t)b.kept * b.R);
        B[q].resize((size_t)b.kept * b.C);
        sv[q].resize(b.kept);
        if (b.kept == 0) continue;
        TNQE_HIP(hipMemcpyAsync(U[q].data(), rb.scratch + b.offU, U[q].size() * 8, hipMemcpyDeviceToHost, st));
        TNQE_HIP(hipMemcpyAsync(B[q].data(), rb.scratch + b.offB, B[q].size() * 8, hipMemcpyDeviceToHost, st));
        TNQE_HIP(hipMemcpyAsync(sv[q].data(), rb.scratch + b.offS, sv[q].size() * 8, hipMemcpyDeviceToHost, st));
      }
      c.sync();
      // the single-site one-hot states (row-major over the expanded site's
      // indices) and the isometry to the two-site one-hot states
      std::vector<double> Tiso;
      int n1 = 0;
      auto add_row = [&]() {
        Tiso.resize(Tiso.size() + n, 0.0);
        return n1++;
      };
      if (site == p) {
        for (int l = 0; l < Dp; ++l)
          for (int kp = 0; kp < 4; ++kp) {
            const int sa = secp[l] / nb1 + qk_a(kp), sb = secp[l] % nb1 + qk_b(kp);
            if (sa > ci.na || sb > ci.nb) continue;
            const int q = blk_of_slot[sa * nb1 + sb];
            if (q < 0) continue;
            const Blk &b = rb.blks[q];
            for (int jj = 0; jj < kept[q]; ++jj) {
              require(sv[q][jj] > 0.0, TNQE_ESINGULAR, "the truncated bond has a vanishing singular value");
              const int m1 = add_row();
              for (int kq = 0; kq < 4; ++kq) {
                const int ra = sa + qk_a(kq), rbb = sb + qk_b(kq);
                if (ra > ci.na || rbb > ci.nb) continue;
                const int r0 = offq(ra, rbb), nr = ci.dim_q(p + 2, 0, ra, rbb);
                for (int r = r0; r < r0 + nr; ++r) {
                  const int m2 = dv.dmap[(((size_t)l * 4 + kp) * 4 + kq) * Dq + r];
                  if (m2 < 0) continue;
                  Tiso[(size_t)m1 * n + m2] = B[q][(size_t)jj * b.C + b.cs[kq] + r - r0] / sv[q][jj];
                }
              }
            }
          }
      } else {
        for (size_t q = 0; q < kept.size(); ++q) {
          const Blk &b = rb.blks[q];
          for (int jj = 0; jj < kept[q]; ++jj)
            for (int kq = 0; kq < 4; ++kq) {
              const int ra = b.sa + qk_a(kq), rbb = b.sb + qk_b(kq);
              if (ra > ci.na || rbb > ci.nb) continue;
              const int r0 = offq(ra, rbb), nr = ci.dim_q(p + 2, 0, ra, rbb);
              for (int r = r0; r < r0 + nr; ++r) {
                const int m1 = add_row();
                for (int kp = 0; kp < 4; ++kp) {
                  const int la = b.sa - qk_a(kp), lb = b.sb - qk_b(kp);
                  if (la < 0 || lb < 0) continue;
                  const int l0 = offp(la, lb), nl = ci.dim_q(p, 0, la, lb);
                  for (int l = l0; l < l0 + nl; ++l) {
                    const int m2 = dv.dmap[(((size_t)l * 4 + kp) * 4 + kq) * Dq + r];
                    if (m2 < 0) continue;
                    Tiso[(size_t)m1 * n + m2] = U[q][(size_t)jj * b.R + b.rs[kp] + l - l0];
                  }
                }
              }
            }
        }
      }
      require(n1 >= 1, TNQE_ESHAPE, "no single-site one-hot states");
      double *dTi = c.upload(Tiso);
      double *P = c.dev<double>((size_t)n1 * n), *Hd1 = c.dev<double>((size_t)n1 * n1);
      double *Sd1 = c.dev<double>((size_t)n1 * n1), *Hc1 = c.dev<double>((size_t)n1 * M);
      double *Sc1 = c.dev<double>((size_t)n1 * M), *tcur = c.dev<double>(n1), *t1 = c.dev<double>(n1);
      sw_gemm(c, kOhPlain, n1, n, n, dTi, Hd2, P);
      sw_gemm(c, kOhPlainBT, n1, n1, n, P, dTi, Hd1);
      sw_gemm(c, kOhPlain, n1, n, n, dTi, Sd2, P);
      sw_gemm(c, kOhPlainBT, n1, n1, n, P, dTi, Sd1);
      sw_gemm(c, kOhPlain, n1, M, n, dTi, Hc2, Hc1);
      sw_gemm(c, kOhPlain, n1, M, n, dTi, Sc2, Sc1);
      sw_gemm(c, kOhPlain, n1, 1, n, dTi, x, tcur);
      const ExpandedRoot er = expanded_root(c, dH, dS, M, ei, n1, Hd1, Sd1, Hc1, Sc1, tcur, 1, tol_ld, eps_S,
                                            max_sweeps, t1, nullptr, nullptr, 0);
      sw_gemm(c, kOhPlainAT, n, 1, n1, dTi, t1, x);    // the updated two-site coefficients
      // TNQE_DEBUG_MITIGATE=1: each round's root and sizes (diagnostics)
      static const bool dbg = std::getenv("TNQE_DEBUG_MITIGATE") != nullptr;
      if (dbg) {
        std::vector<double> hx(n), hc(n1);
        TNQE_HIP(hipMemcpyAsync(hx.data(), x, n * sizeof(double), hipMemcpyDeviceToHost, st));
        TNQE_HIP(hipMemcpyAsync(hc.data(), tcur, n1 * sizeof(double), hipMemcpyDeviceToHost, st));
        c.sync();
        double nx = 0.0, nc = 0.0;
        for (double v : hx) nx += v * v;
        for (double v : hc) nc += v * v;
        std::fprintf(stderr, "mitigation rep %d site %d: n1 %d columns %d kept %d E %.15f |x'|^2 %.15f |t_cur|^2 %.15f\n",
                     rep, site, n1, er.D, er.n_kept, er.E, nx, nc);
      }
      mo.E = er.E;
      mo.columns = er.D;
      mo.kept = er.n_kept;
      if (rep == nreps - 1 && site == p + 1) {
        // A_p = Q (the fixed left site), A_{p+1} = the updated site
        std::vector<double> h1(n1);
        TNQE_HIP(hipMemcpyAsync(h1.data(), t1, n1 * sizeof(double), hipMemcpyDeviceToHost, st));
        c.sync();
        std::fill(Ap.begin(), Ap.end(), 0.0);
        std::fill(Aq.begin(), Aq.end(), 0.0);
        int m1 = 0;
        for (size_t q = 0; q < kept.size(); ++q) {
          const Blk &b = rb.blks[q];
          for (int jj = 0; jj < kept[q]; ++jj) {
            const int j = j0[q] + jj;
            for (int kp = 0; kp < 4; ++kp) {
              const int la = b.sa - qk_a(kp), lb = b.sb - qk_b(kp);
              if (la < 0 || lb < 0) continue;
              const int l0 = offp(la, lb), nl = ci.dim_q(p, 0, la, lb);
              for (int l = l0; l < l0 + nl; ++l)
                Ap[((size_t)l * 4 + kp) * Dn + j] = U[q][(size_t)jj * b.R + b.rs[kp] + l - l0];
            }
            for (int kq = 0; kq < 4; ++kq) {
              const int ra = b.sa + qk_a(kq), rbb = b.sb + qk_b(kq);
              if (ra > ci.na || rbb > ci.nb) continue;
              const int r0 = offq(ra, rbb), nr = ci.dim_q(p + 2, 0, ra, rbb);
              for (int r = r0; r < r0 + nr; ++r) Aq[((size_t)j * 4 + kq) * Dq + r] = h1[m1++];
            }
          }
        }
      }
      c.ctx->pool.rewind(mk);
    }
  }
  return mo;
}

void sweep_one(tnqe_ctx *ctx, tnqe_problem &pb, const tnqe_options &op, const tnqe_sweep_options &so, int ei, int p,
               const double *H, const double *S, SweepOut &out, tnqe_report &rep) {
  Call c{ctx};
  const auto t0 = Clock::now();
  hipStream_t st = ctx->stream;
  const int M = pb.M, N = pb.N, nslot = pb.nslot();
  require(M <= kMaxM, TNQE_ESHAPE, "more than 32 states");
  const int chi_cap = op.chi_cap_override > 0 ? op.chi_cap_override : op.chi;
  const int max_sweeps = op.max_sweeps > 0 ? op.max_sweeps : 40;
  const double eps_S = op.eps_S > 0 ? op.eps_S : 1e-12;
  const double tol_ld = so.tol_ld > 0 ? so.tol_ld : 1e-3;
  const int n_grid = so.n_grid > 0 ? so.n_grid : 36, n_golden = so.n_golden >= 0 ? so.n_golden : 40;
  require(so.rotation >= TNQE_ROT_NONE && so.rotation <= TNQE_ROT_GIVENS, TNQE_EINVAL, "unknown rotation type");
  require(n_grid % 2 == 0, TNQE_EINVAL, "n_grid must be even (the grid holds theta = 0)");
  require(so.nreps >= 0 && so.nreps <= 64, TNQE_EINVAL, "nreps out of range");
  // current pencil and its lowest root
  std::vector<double> hH(H, H + (size_t)M * M), hS(S, S + (size_t)M * M);
  for (double v : hH) require(std::isfinite(v), TNQE_ENONFINITE, "non-finite pencil element");
  for (double v : hS) require(std::isfinite(v), TNQE_ENONFINITE, "non-finite pencil element");
  double *dH = c.upload(hH), *dS = c.upload(hS);
  {
    std::vector<int> Ms{M};
    std::vector<int64_t> offs{0};
    double *dout = c.dev<double>(8 + kMaxM);
    launch_gep(dH, dS, c.upload(Ms), c.upload(offs), 1, eps_S, dout, st);
    std::vector<double> g(8 + kMaxM);
    TNQE_HIP(hipMemcpyAsync(g.data(), dout, g.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    c.sync();
    require(g[5] == 0.0, TNQE_ESINGULAR, "the current pencil has no positive overlap eigenvalue");
    out.E_old = g[0];
  }
  // 1. expanded pencil blocks; state ei centred on (p, p+1)
  OneHotDev dv;
  onehot_core(c, pb, op, ei, p, dv, rep);
  KetSet &ci = dv.ci;
  const int n = (int)dv.index.size(), D = n + M - 1;
  out.n = n;
  out.D = D;
  require(D <= 1024, TNQE_ESHAPE, "expanded pencil wider than 1024 columns");
  const auto tg = Clock::now();
  // 2-5. discard, expanded root, parameter update into the dense two-site
  // tensor T[l][k_p][k_{p+1}][r]
  const int Dp = dv.Dp, Dq = dv.Dq;
  const int64_t tsize = (int64_t)Dp * 16 * Dq;
  double *dT = c.dev<double>(tsize), *dtn = c.dev<double>(n);
  {
    const ExpandedRoot er = expanded_root(c, dH, dS, M, ei, n, dv.Hd, dv.Sd, dv.Hc, dv.Sc, dv.Sc + ei, M, tol_ld,
                                          eps_S, max_sweeps, dtn, dv.d_dense, dT, tsize);
    out.E1 = er.E;
    out.n_kept = er.n_kept;
    out.n_dropped_S = er.n_dropped_S;
  }
  out.E_new = out.E1;
  out.tnew.resize(n);
  TNQE_HIP(hipMemcpyAsync(out.tnew.data(), dtn, n * sizeof(double), hipMemcpyDeviceToHost, st));
  c.sync();
  rep.t_gep_ms = ms_since(tg);
  // 6. rotation of the bond (nothing to gain when xi(0) is below the
  // tolerance: xi is not negative, so no rotation lowers it by more)
  const Gate16 ident = givens_gate(0.0);
  Gate16 chosen = ident;
  out.xi_none = out.xi = truncation_errors(c, ci, p, dT, {ident}, chi_cap, max_sweeps)[0];
  if (so.rotation == TNQE_ROT_NONE || out.xi_none < kXiTol) {
  } else if (so.rotation == TNQE_ROT_FSWAP) {
    const Gate16 f = fswap_gate();
    const double xs = truncation_errors(c, ci, p, dT, {f}, chi_cap, max_sweeps)[0];
    if (xs < out.xi_none - kXiTol) {
      out.theta = M_PI / 2;
      out.xi = xs;
      chosen = f;
    }
  } else {
    // theta_opt: the grid, then golden-section steps on one spacing either
    // side of its best point
    std::vector<Gate16> gg;
    std::vector<double> grid(n_grid);
    for (int q = 0; q < n_grid; ++q) {
      grid[q] = (double)(q - n_grid / 2) * (M_PI / n_grid);
      gg.push_back(givens_gate(grid[q]));
    }
    const std::vector<double> vals = truncation_errors(c, ci, p, dT, gg, chi_cap, max_sweeps);
    int qb = 0;
    for (int q = 1; q < n_grid; ++q)
      if (vals[q] < vals[qb]) qb = q;
    const double xi0 = vals[n_grid / 2];
    auto f = [&](double th) { return truncation_errors(c, ci, p, dT, {givens_gate(th)}, chi_cap, max_sweeps)[0]; };
    const double h = M_PI / n_grid, gr = (std::sqrt(5.0) - 1.0) / 2.0;
    double a = grid[qb] - h, b = grid[qb] + h;
    double x1 = b - gr * (b - a), x2 = a + gr * (b - a);
    double f1 = f(x1), f2 = f(x2);
    for (int it = 0; it < n_golden; ++it) {
      if (f1 <= f2) {
        b = x2;
        x2 = x1;
        f2 = f1;
        x1 = b - gr * (b - a);
        f1 = f(x1);
      } else {
        a = x1;
        x1 = x2;
        f1 = f2;
        x2 = a + gr * (b - a);
        f2 = f(x2);
      }
    }
    double th = f1 <= f2 ? x1 : x2, fv = f1 <= f2 ? f1 : f2;
    if (vals[qb] < fv) {
      th = grid[qb];
      fv = vals[qb];
    }
    if (!(fv < xi0 - kXiTol)) {
      th = 0.0;
      fv = xi0;
    }
    out.theta = th;
    out.xi = fv;
    chosen = givens_gate(th);
  }
  // 7. truncation of the rotated tensor (rule of the gates) and the new sites
  RotatedBlocks rb;
  rotated_blocks(c, ci, p, dT, {chosen}, max_sweeps, rb);
  std::vector<std::vector<double>> sv(rb.blks.size());
  for (size_t q = 0; q < rb.blks.size(); ++q) {
    sv[q].resize(rb.blks[q].n);
    TNQE_HIP(hipMemcpyAsync(sv[q].data(), rb.scratch + rb.blks[q].offS, sv[q].size() * sizeof(double),
                            hipMemcpyDeviceToHost, st));
  }
  c.sync();
  std::vector<double> all;
  std::vector<int> owner;
  for (size_t q = 0; q < sv.size(); ++q)
    for (double v : sv[q]) {
      all.push_back(v);
      owner.push_back((int)q);
    }
  double total = 0.0;
  for (double v : all) total += v * v;
  int nnz = 0;
  for (double v : all) nnz += v * v > op.tau_w * total ? 1 : 0;
  const int keep_n = std::min(chi_cap, nnz);
  std::vector<int> order(all.size());
  for (size_t q = 0; q < order.size(); ++q) order[q] = (int)q;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return all[x] > all[y]; });
  std::vector<int> kept(rb.blks.size(), 0);
  double kept_w = 0.0;
  for (int q = 0; q < keep_n; ++q) {
    kept[owner[order[q]]]++;
    kept_w += all[order[q]] * all[order[q]];
  }
  out.discarded = 0.0;
  for (int q = keep_n; q < (int)order.size(); ++q) out.discarded += all[order[q]] * all[order[q]];
  (void)kept_w;
  for (size_t q = 0; q < rb.blks.size(); ++q) rb.blks[q].kept = kept[q];
  {
    Blk *dblk = c.upload(rb.blks);
    const std::vector<int> uf = unit_prefix(rb.blks, [](const Blk &b) { return factor_units(b); });
    const int *duf = c.upload(uf);
    launch_svd_factor(dblk, Units{duf, (int)rb.blks.size(), uf.back()}, rb.scratch, st);
    c.check_launch();
  }
  std::vector<std::vector<double>> Uh(rb.blks.size()), Bh(rb.blks.size());
  for (size_t q = 0; q < rb.blks.size(); ++q) {
    const Blk &b = rb.blks[q];
    Uh[q].resize((size_t)b.kept * b.R);
    Bh[q].resize((size_t)b.kept * b.C);
    if (b.kept == 0) continue;
    TNQE_HIP(hipMemcpyAsync(Uh[q].data(), rb.scratch + b.offU, Uh[q].size() * sizeof(double), hipMemcpyDeviceToHost, st));
    TNQE_HIP(hipMemcpyAsync(Bh[q].data(), rb.scratch + b.offB, Bh[q].size() * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  // the canonical sites of state ei
  std::vector<std::vector<double>> site(N);
  for (int x = 0; x < N; ++x) {
    site[x].resize((size_t)ci.htot[x] * 4 * ci.htot[x + 1]);
    TNQE_HIP(hipMemcpyAsync(site[x].data(), ci.site_ptr[x], site[x].size() * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  c.sync();
  const int Dn = keep_n;
  out.new_bond = Dn;
  std::vector<double> Ap((size_t)Dp * 4 * Dn, 0.0), Aq((size_t)Dn * 4 * Dq, 0.0);
  std::vector<int32_t> newq;
  {
    auto offp = [&](int a, int b2) { return ci.off_q(p, 0, a, b2); };
    auto offq = [&](int a, int b2) { return ci.off_q(p + 2, 0, a, b2); };
    int j0 = 0;
    for (size_t q = 0; q < rb.blks.size(); ++q) {
      const Blk &b = rb.blks[q];
      for (int j = 0; j < b.kept; ++j) {
        newq.push_back(b.sa);
        newq.push_back(b.sb);
        for (int row = 0; row < b.R; ++row) {
          int kp = 0;
          while (row >= b.rs[kp + 1]) ++kp;
          const int l = offp(b.sa - qk_a(kp), b.sb - qk_b(kp)) + row - b.rs[kp];
          Ap[((size_t)l * 4 + kp) * Dn + j0 + j] = Uh[q][(size_t)j * b.R + row];
        }
        for (int cl = 0; cl < b.C; ++cl) {
          int kq = 0;
          while (cl >= b.cs[kq + 1]) ++kq;
          const int rr = offq(b.sa + qk_a(kq), b.sb + qk_b(kq)) + cl - b.cs[kq];
          Aq[((size_t)(j0 + j) * 4 + kq) * Dq + rr] = Bh[q][(size_t)j * b.C + cl];
        }
      }
      j0 += b.kept;
    }
  }
  // single-site mitigation (App. A4)
  if (so.nreps > 0) {
    std::vector<int> kept_blk(rb.blks.size());
    for (size_t q = 0; q < rb.blks.size(); ++q) kept_blk[q] = rb.blks[q].kept;
    const MitOut mo = mitigate(c, ci, p, dv, chosen, dH, dS, M, ei, kept_blk, so.nreps, tol_ld, eps_S, max_sweeps,
                               Ap, Aq, Dn);
    out.E_new = mo.E;
    out.mit_columns = mo.columns;
    out.mit_kept = mo.kept;
  }
  out.accepted = out.E_new < out.E_old + so.e_tol ? 1 : 0;
  site[p] = std::move(Ap);
  site[p + 1] = std::move(Aq);
  out.bond_dim.assign(N + 1, 0);
  out.bond_qn.clear();
  for (int bd = 0; bd <= N; ++bd) {
    if (bd == p + 1) {
      out.bond_dim[bd] = Dn;
      out.bond_qn.insert(out.bond_qn.end(), newq.begin(), newq.end());
      continue;
    }
    out.bond_dim[bd] = ci.htot[bd];
    for (int s2 = 0; s2 < nslot; ++s2)
      for (int d = 0; d < ci.dim(bd, 0, s2); ++d) {
        out.bond_qn.push_back(s2 / (pb.nb + 1));
        out.bond_qn.push_back(s2 % (pb.nb + 1));
      }
  }
  out.sites.clear();
  for (int x = 0; x < N; ++x) out.sites.insert(out.sites.end(), site[x].begin(), site[x].end());
  // 8. merge: g4(theta) on the sites is G(R_p(theta)), compensated by
  // U <- U R_p(theta)^T; the FSWAP is G(P) with P exchanging p and p+1
  out.U = pb.mps[ei].U;
  if (out.theta != 0.0) {
    std::vector<double> &U = out.U;
    if (so.rotation == TNQE_ROT_FSWAP) {
      for (int r2 = 0; r2 < N; ++r2) std::swap(U[(size_t)r2 * N + p], U[(size_t)r2 * N + p + 1]);
    } else {
      const double cth = std::cos(out.theta), sth = std::sin(out.theta);
      for (int r2 = 0; r2 < N; ++r2) {
        const double u0 = U[(size_t)r2 * N + p], u1 = U[(size_t)r2 * N + p + 1];
        U[(size_t)r2 * N + p] = cth * u0 + sth * u1;
        U[(size_t)r2 * N + p + 1] = -sth * u0 + cth * u1;
      }
    }
  }
  rep.t_total_ms = ms_since(t0);
}

// Upper bound of the device memory one solve takes from its pool (bytes):
// the problem's site tensors, the MPO coefficients and structure, the two
// ket sets, and the larger of the gate phase's and the environment phase's
// peaks, each for the largest bond dimensions truncation can produce (the
// bond capacities, and per quantum-number sector the exact sector dimension
// capped by them).  Blocks of a two-site or one-site matrix partition its
// rows and columns, so a step's per-block storage is bounded by that of the
// whole matrix; the environment layout is planned for the bounding sector
// dimensions, and its sizes grow with every dimension.
size_t workspace_bound(tnqe_ctx *ctx, const tnqe_problem &pb, const tnqe_options &op) {
  auto a256 = [](double bytes) { return (size_t)((std::max(1.0, bytes) + 255.0) / 256.0) * 256; };
  const int N = pb.N, M = pb.M, nslot = pb.nslot();
  const int P = M * (M - 1) / 2, npair = M * (M + 1) / 2;
  const int chi_cap = op.chi_cap_override > 0 ? op.chi_cap_override : op.chi;
  const MpoStructure &mpo = mpo_for(ctx, N);
  const int64_t nnz = mpo.site_nnz_off[N];
  size_t persistent = 0;
  int64_t sites = 0;
  for (int i = 0; i < M; ++i)
    for (int p = 0; p < N; ++p) sites += (int64_t)pb.mps[i].dims[p] * 4 * pb.mps[i].dims[p + 1];
  persistent += a256(8.0 * sites) + a256(8.0 * nnz * M);
  int64_t nrp = 1, ncl = 1;
  for (int x = 0; x < N; ++x)
    for (const MpoGroup &g : mpo.groups[x]) {
      nrp += (int64_t)g.rowptr.size();
      ncl += (int64_t)g.col.size();
    }
  persistent += a256(4.0 * nrp) + a256(4.0 * ncl);
  const std::vector<int> cap = bond_caps(pb, chi_cap);
  int64_t stride = 0;
  for (int p = 0; p < N; ++p) stride = std::max(stride, ((int64_t)cap[p] * 4 * cap[p + 1] + 31) & ~int64_t(31));
  auto ketset = [&](int n) {
    return a256(8.0 * (N + 1) * n * nslot) + a256(4.0 * (N + 1) * n) + a256(8.0 * stride * (N + 1) * n) +
           a256(8.0 * n * N);
  };
  const double blk = sizeof(Blk);
  // run_svd: one index list per (kernel, threads) group, the sweep counters
  auto svd_tables = [&](double nblk) { return 42 * 256.0 + 4.0 * nblk + a256(4.0 * nblk); };
  // per ket: T, U, B, S (and the global Jacobi work area) of blocks that
  // partition an R_tot x C_tot matrix, 32-double granules per piece
  auto block_scratch = [&](double Rt, double Ct) { return 8.0 * (4.0 * Rt * Ct + 2.0 * std::min(Rt, Ct) + 160.0 * nslot); };
  auto move_bound = [&](int n, double Rt, double Ct, double old_site) {
    const double nblk = (double)n * nslot;
    return a256(n * block_scratch(Rt, Ct)) + a256(8.0 * old_site * n) + 4 * a256(8.0 * n) + a256(blk * nblk) +
           3 * a256(4.0 * (nblk + 1)) + svd_tables(nblk);
  };
  size_t gates_peak = 0;
  if (P > 0) {
    persistent += ketset(M) + ketset(P);
    for (int p = 0; p + 1 < N; ++p)   // canonicalisation (QR moves right)
      gates_peak = std::max(gates_peak, (size_t)move_bound(M, 4.0 * cap[p], cap[p + 1],
                                                           (double)cap[p + 1] * 4 * cap[p + 2]) +
                                            3 * a256(8.0 * M));
    gates_peak = std::max(gates_peak, 3 * a256(8.0 * P) + a256(4.0 * P));
    for (int a = 0; a + 1 < N; ++a) {
      // centre moves into site a + 1 (LQ from the right) or a (QR from the left)
      const double lq = move_bound(P, cap[a + 1], 4.0 * cap[a + 2], 0.0);
      const double qr = move_bound(P, 4.0 * cap[a], cap[a + 1], (double)cap[a + 1] * 4 * cap[a + 2]);
      const double Rt = 4.0 * cap[a], Ct = 4.0 * cap[a + 2], nblk = (double)P * nslot;
      const double step = a256(P * (block_scratch(Rt, Ct) + 8.0 * (Rt * Ct + 32.0 * nslot))) + a256(8.0 * 256 * P) +
                          a256(4.0 * nblk) + a256(8.0 * 3 * P) + a256(16.0 * P) + 2 * a256(blk * nblk) +
                          a256(4.0 * P * nslot) + 4 * a256(4.0 * (nblk + 1)) + a256(4.0 * (P + 1)) + svd_tables(nblk);
      gates_peak = std::max(gates_peak, (size_t)std::max(step, std::max(lq, qr)));
    }
  }
  // environment phase, for the bounding sector dimensions of every bond
  std::vector<std::vector<int>> dpad(N + 1, std::vector<int>(nslot, 0));
  for (int b = 0; b <= N; ++b)
    for (int a = 0; a <= pb.na; ++a)
      for (int bb = 0; bb <= pb.nb; ++bb) {
        const int s = a * (pb.nb + 1) + bb;
        double ex = std::min(binom(b, a) * binom(b, bb), binom(N - b, pb.na - a) * binom(N - b, pb.nb - bb));
        int mx = 0;
        for (int i = 0; i < M; ++i) mx = std::max(mx, pb.mps[i].secdim[b][s]);
        dpad[b][s] = (int)std::min<double>(cap[b], std::max<double>(ex, mx));
      }
  EnvLayout lay;
  plan_env_layout(mpo, nullptr, N, pb.na, pb.nb, dpad, host_pool(ctx), lay);
  const double eb = op.precision == TNQE_FP64 ? 8.0 : 4.0;
  const int nitem = M + P;
  double env = a256(8.0 * nitem * (N + 1) * nslot) + a256(4.0 * nitem * (N + 1));
  if (op.precision != TNQE_FP64) {
    double tot = 0.0;
    for (int p = 0; p < N; ++p) tot += (double)cap[p] * 4 * cap[p + 1];
    env += a256(4.0 * tot * nitem) + 3 * a256(8.0 * nitem * N) + a256(4.0 * nnz * M);
  }
  // when the common layout does not fit, every pair runs alone in a layout of
  // its own two items: per sector at most min(cap, bounding dimension), and
  // at most 2 cap over the sectors of a bond
  const auto &cls = mpo.classes;
  auto dB = [&](int bnd, int a, int bb) {
    return (a < 0 || bb < 0 || a > pb.na || bb > pb.nb) ? 0.0 : (double)dpad[bnd][a * (pb.nb + 1) + bb];
  };
  auto pairsum = [&](int b1, int da1, int db1, int b2, int da2, int db2) {   // sum_s d1(s + d1) d2(s + d2)
    double acc = 0.0;
    for (int a = -2; a <= pb.na + 2; ++a)
      for (int bb = -2; bb <= pb.nb + 2; ++bb) acc += dB(b1, a + da1, bb + db1) * dB(b2, a + da2, bb + db2);
    return acc;
  };
  double Lmax = 1, Xmax = 1, Ymax = 1;
  for (int bnd = 0; bnd <= N; ++bnd) {
    double l = 0.0;
    for (const MpoClass &c : cls[bnd])
      l += c.nw * std::min(4.0 * cap[bnd] * cap[bnd], pairsum(bnd, c.da, c.db, bnd, 0, 0));
    Lmax = std::max(Lmax, l);
  }
  for (int x = 0; x < N; ++x) {
    const double box = 4.0 * cap[x] * cap[x + 1];
    double xs = 0.0, ys = 0.0;
    for (const MpoClass &c : cls[x])
      for (int k = 0; k < 4; ++k) xs += c.nw * std::min(box, pairsum(x, c.da, c.db, x + 1, qk_a(k), qk_b(k)));
    for (const MpoClass &c : cls[x + 1])
      for (int k = 0; k < 4; ++k) ys += c.nw * std::min(box, pairsum(x, c.da - qk_a(k), c.db - qk_b(k), x + 1, 0, 0));
    Xmax = std::max(Xmax, xs);
    Ymax = std::max(Ymax, ys);
  }
  int64_t ndesc = 0;
  for (int x = 0; x < N; ++x) {
    const EnvSiteTabs &t = lay.tabs[x];
    env += a256((double)sizeof(EnvG1) * t.g1.size()) + a256((double)sizeof(EnvG2) * t.g2.size()) +
           a256((double)sizeof(MixTask) * t.tasks.size()) + a256((double)sizeof(MixSrc) * t.srcs.size()) +
           a256((double)sizeof(EnvFinal) * t.fin.size());
    ndesc += (int64_t)t.g1.size() + t.tasks.size() + t.g2.size();
    for (auto &lv : t.dense) {
      env += a256((double)sizeof(EnvGD) * lv.size());
      ndesc += (int64_t)lv.size();
    }
  }
  // one pair, with the allowance the batching keeps free for its tables
  env += 2 * a256(eb * Lmax) + a256(eb * Xmax) + a256(eb * Ymax) + (double)ndesc * sizeof(EnvWork) +
         (2.0 * N + 12) * sizeof(void *) + 256.0 * (5 * N + 24) + 64.0 * (ndesc + 64) + 256.0 * (6 * N + 24);
  // mixed precision runs the FP64 pairs first, then the FP32 ones
  (void)npair;
  const size_t gep = 4 * a256(8.0 * M * M) + a256(8.0 * (8 + kMaxM)) + 2 * a256(8.0);
  const size_t peak = std::max<size_t>(gates_peak, (size_t)env) + gep;
  const size_t total = persistent + peak;
  return total + total / 16 + (16u << 20);
}
}  // namespace
}  // namespace tnqe

// ============================================================== C ABI
using namespace tnqe;

namespace {

tnqe_status fail(tnqe_ctx *ctx, tnqe_status st, const std::string &msg) {
  if (ctx) ctx->last_error = msg;
  return st;
}

// Wait for everything the context has queued (main and side streams, errors
// ignored) so that memory handed out during a failed call can be reused.
void quiesce(tnqe_ctx *ctx) {
  if (!ctx->aux[0]) return;   // a host-only context has queued nothing
  (void)hipStreamSynchronize(ctx->stream);
  for (int i = 0; i < tnqe_ctx::kAux; ++i)
    if (ctx->aux[i]) (void)hipStreamSynchronize(ctx->aux[i]);
  (void)hipGetLastError();
}

template <class F>
tnqe_status guarded(tnqe_ctx *ctx, F &&f) {
  try {
    f();
    if (ctx) ctx->last_error.clear();
    return TNQE_OK;
  } catch (const Error &e) {
    if (ctx) {
      quiesce(ctx);
      ctx->pool.release_all();
      ctx->staging.reset();
    }
    return fail(ctx, e.st, e.what());
  } catch (const std::bad_alloc &) {
    if (ctx) {
      quiesce(ctx);
      ctx->pool.release_all();
      ctx->staging.reset();
    }
    return fail(ctx, TNQE_ENOMEM, "host allocation failed");
  } catch (const std::exception &e) {
    if (ctx) {
      quiesce(ctx);
      ctx->pool.release_all();
      ctx->staging.reset();
    }
    return fail(ctx, TNQE_EINVAL, e.what());
  }
}

}  // namespace

namespace {

// Host-side validation and copies of a problem (no device work): shapes,
// |U^T U - I|_max <= 1e-10, zero entries outside particle-number blocks,
// finite values, every MPS in the (n_alpha, n_beta) sector, M <= kMaxM.
void load_problem(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps, tnqe_problem *pb) {
  require(M >= 1 && M <= kMaxM, TNQE_EINVAL, "M must be in [1, " + std::to_string(kMaxM) + "]");
  const int N = ham->N;
  require(N >= 1 && N <= 64, TNQE_ESHAPE, "N must be in [1, 64]");
  require(ham->n_alpha >= 0 && ham->n_alpha <= N && ham->n_beta >= 0 && ham->n_beta <= N, TNQE_ESHAPE,
          "electron counts out of range");
  require(ham->h != nullptr, TNQE_EINVAL, "h is NULL");
  require((ham->n_chol > 0 && ham->L) || (ham->n_chol == 0 && ham->g), TNQE_EINVAL,
          "two-electron integrals missing");
  pb->N = N;
  pb->na = ham->n_alpha;
  pb->nb = ham->n_beta;
  pb->M = M;
  pb->e_core = ham->e_core;
  require(std::isfinite(pb->e_core), TNQE_ENONFINITE, "e_core not finite");
  const size_t N2 = (size_t)N * N;
  pb->h.assign(ham->h, ham->h + N2);
  for (size_t x = 0; x < N2; ++x) {
    require(std::isfinite(pb->h[x]), TNQE_ENONFINITE, "h has a non-finite entry");
    require(std::fabs(pb->h[x] - pb->h[(x % N) * N + x / N]) <= 1e-12 * (1 + std::fabs(pb->h[x])),
            TNQE_EINVAL, "h is not symmetric");
  }
  if (ham->n_chol > 0) {
    pb->K = ham->n_chol;
    pb->L.assign(ham->L, ham->L + (size_t)pb->K * N2);
    for (double v : pb->L) require(std::isfinite(v), TNQE_ENONFINITE, "L has a non-finite entry");
    pb->g.clear();
  } else {
    pb->K = 0;
    pb->g.assign(ham->g, ham->g + N2 * N2);
    for (double v : pb->g) require(std::isfinite(v), TNQE_ENONFINITE, "g has a non-finite entry");
  }
  const int nslot = pb->nslot();
  int64_t total = 0;
  pb->mps.resize(M);
  // bond labels per MPS, kept for the scan of the site tensors, which runs
  // on the host workers (the labels and U are checked serially first)
  std::vector<std::vector<std::vector<int>>> lab_a(M), lab_b(M);
  for (int i = 0; i < M; ++i) {
    const tnqe_mps &m = mps[i];
    require(m.bond_dim && m.bond_qn && m.sites && m.U, TNQE_EINVAL, "MPS field is NULL");
    auto &pm = pb->mps[i];
    pm.dims.assign(m.bond_dim, m.bond_dim + N + 1);
    require(pm.dims[0] == 1 && pm.dims[N] == 1, TNQE_ESHAPE, "boundary bonds must have dimension 1");
    pm.secdim.assign(N + 1, std::vector<int>(nslot, 0));
    std::vector<std::vector<int>> qa(N + 1), qb(N + 1);
    int64_t qo = 0;
    for (int b = 0; b <= N; ++b) {
      require(pm.dims[b] >= 1 && pm.dims[b] <= 1 << 20, TNQE_ESHAPE, "bond dimension out of range");
      int prev = -1;
      for (int x = 0; x < pm.dims[b]; ++x) {
        const int a = m.bond_qn[2 * (qo + x)], bb = m.bond_qn[2 * (qo + x) + 1];
        require(a >= 0 && a <= pb->na && bb >= 0 && bb <= pb->nb, TNQE_EQN, "bond label out of range");
        const int s = a * (pb->nb + 1) + bb;
        require(s >= prev, TNQE_EQN, "bond indices not sorted by sector");
        prev = s;
        pm.secdim[b][s]++;
        qa[b].push_back(a);
        qb[b].push_back(bb);
      }
      qo += pm.dims[b];
    }
    require(qa[0][0] == 0 && qb[0][0] == 0 && qa[N][0] == pb->na && qb[N][0] == pb->nb, TNQE_EQN,
            "MPS is not in the (n_alpha, n_beta) sector");
    pm.U.assign(m.U, m.U + N2);
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) {
        double acc = 0.0;
        for (int p = 0; p < N; ++p) acc += pm.U[p * N + a] * pm.U[p * N + b];
        require(std::isfinite(acc), TNQE_ENONFINITE, "U has a non-finite entry");
        require(std::fabs(acc - (a == b ? 1.0 : 0.0)) <= 1e-10, TNQE_ENOTORTH, "U is not orthogonal");
      }
    pm.site_off.resize(N);
    for (int p = 0; p < N; ++p) {
      pm.site_off[p] = total;
      total += (int64_t)pm.dims[p] * 4 * pm.dims[p + 1];
    }
    lab_a[i] = std::move(qa);
    lab_b[i] = std::move(qb);
  }
  // site tensors: finite, and nonzero only inside their particle-number
  // blocks (one MPS per worker)
  host_pool(ctx).parallel_for(M, [&](int i) {
    const auto &pm = pb->mps[i];
    const auto &qa = lab_a[i], &qb = lab_b[i];
    const double *sp = mps[i].sites;
    for (int p = 0; p < N; ++p) {
      const int dl = pm.dims[p], dr = pm.dims[p + 1];
      for (int l = 0; l < dl; ++l)
        for (int k = 0; k < 4; ++k)
          for (int r = 0; r < dr; ++r) {
            const double v = sp[((int64_t)l * 4 + k) * dr + r];
            require(std::isfinite(v), TNQE_ENONFINITE, "site tensor has a non-finite entry");
            if (v != 0.0)
              require(qa[p + 1][r] == qa[p][l] + (k & 1) && qb[p + 1][r] == qb[p][l] + (k >> 1), TNQE_EQN,
                      "site tensor entry outside its particle-number block");
          }
      sp += (int64_t)dl * 4 * dr;
    }
  });
}

// Site tensors of every MPS to device memory: a buffer the problem owns, or
// (calls working in a caller's workspace) the context's arena.
void place_sites(tnqe_ctx *ctx, tnqe_problem *pb, const tnqe_mps *mps) {
  int64_t total = 0;
  for (const auto &m : pb->mps)
    for (int p = 0; p < pb->N; ++p) total += (int64_t)m.dims[p] * 4 * m.dims[p + 1];
  pb->device = ctx->device;
  if (ctx->pool.arena()) {
    pb->d_sites = static_cast<double *>(ctx->pool.get(std::max<int64_t>(1, total) * sizeof(double)));
    pb->owns_sites = false;
  } else {
    TNQE_HIP(hipMalloc(&pb->d_sites, std::max<int64_t>(1, total) * sizeof(double)));
    pb->owns_sites = true;
  }
  int64_t o = 0;
  for (int i = 0; i < pb->M; ++i) {
    int64_t n = 0;
    for (int p = 0; p < pb->N; ++p) n += (int64_t)pb->mps[i].dims[p] * 4 * pb->mps[i].dims[p + 1];
    TNQE_HIP(hipMemcpy(pb->d_sites + o, mps[i].sites, n * sizeof(double), hipMemcpyHostToDevice));
    o += n;
  }
}

void free_sites(tnqe_problem *pb) {
  if (pb->d_sites && pb->owns_sites) {
    (void)hipSetDevice(pb->device);
    (void)hipFree(pb->d_sites);
  }
  pb->d_sites = nullptr;
}

tnqe_status check_options(tnqe_ctx *ctx, const tnqe_options *o) {
  if (o->precision < TNQE_FP64 || o->precision > TNQE_ENV_BF16X3)
    return fail(ctx, TNQE_EINVAL, "unknown precision mode");
  if ((o->chi_cap_override > 0 ? o->chi_cap_override : o->chi) < 1) return fail(ctx, TNQE_EINVAL, "chi must be >= 1");
  if (o->autotune < 0 || o->autotune >= 2 + kTileCands) return fail(ctx, TNQE_EINVAL, "unknown tile mode");
  return TNQE_OK;
}

// The caller's workspace as the pool's arena for the length of one call.
struct ArenaScope {
  tnqe_ctx *ctx;
  bool on;
  ArenaScope(tnqe_ctx *c, void *ws, size_t bytes, bool no_alloc) : ctx(c), on(ws != nullptr) {
    if (on) ctx->pool.set_arena(ws, bytes);
    ctx->no_alloc = no_alloc;
    ctx->staging.allow_pinned_growth(!no_alloc);
  }
  ~ArenaScope() {
    if (on) ctx->pool.clear_arena();
    ctx->no_alloc = false;
    ctx->staging.allow_pinned_growth(true);
    ctx->mpo_dev_call.reset();
  }
};

// One subspace from host inputs: validation, sites to device memory, solve.
// With a workspace every device buffer of the call lies in it.
tnqe_status subspace_call(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                          const tnqe_options *opts, void *ws, size_t ws_bytes, bool no_alloc, SolveOut &so) {
  tnqe_problem pb;
  tnqe_status st = guarded(ctx, [&] {
    TNQE_HIP(hipSetDevice(ctx->device));
    load_problem(ctx, ham, M, mps, &pb);
    ArenaScope scope(ctx, ws, ws_bytes, no_alloc);
    try {
      place_sites(ctx, &pb, mps);
      solve_one(ctx, pb, *opts, so);
      if (ws) so.rep.ws_peak_bytes = (double)ctx->pool.arena_peak();
      ctx->pool.release_all();
    } catch (...) {
      // nothing of this call may still run when the workspace goes back
      quiesce(ctx);
      ctx->pool.release_all();
      ctx->staging.reset();
      free_sites(&pb);
      throw;
    }
  });
  free_sites(&pb);
  return st;
}

// Independent subspaces run concurrently: up to kBatchWorkers worker
// contexts on the same device, each with its own stream (default priority),
// side streams, device pool and two host helper threads, take subspaces in
// decreasing order of estimated cost; the GPU is shared by their launches.
// tnqe_options.workers of the first subspace, else TNQE_BATCH_WORKERS, sets
// the count (1: one after another).
constexpr int kBatchWorkers = 4;

int batch_workers(int n, const tnqe_options &o) {
  static const int env = [] {
    const char *e = std::getenv("TNQE_BATCH_WORKERS");
    return e ? std::max(1, std::atoi(e)) : kBatchWorkers;
  }();
  return std::max(1, std::min(n, o.workers > 0 ? o.workers : env));
}

tnqe_ctx *worker(tnqe_ctx *ctx, int w) {
  while ((int)ctx->sub.size() <= w) {
    tnqe_ctx *sw = nullptr;
    if (tnqe_create(&sw, ctx->device, nullptr) != TNQE_OK) throw Error(TNQE_EHIP, "cannot create a batch worker");
    if (hipStreamCreateWithFlags(&sw->own_stream, hipStreamNonBlocking) != hipSuccess) {
      tnqe_destroy(sw);
      throw Error(TNQE_EHIP, "cannot create a batch worker stream");
    }
    sw->stream = sw->own_stream;
    sw->host_workers = 2;
    ctx->sub.push_back(sw);
  }
  return ctx->sub[w];
}

// Runs run(worker context, worker index, s) for s in order (cost-sorted by
// the caller) on W workers; returns each subspace's status.  The workers'
// streams first wait for work queued on the caller's stream.
std::vector<tnqe_status> run_batch(tnqe_ctx *ctx, const std::vector<int> &order, int W,
                                   const std::function<tnqe_status(tnqe_ctx *, int, int)> &run) {
  const int n = (int)order.size();
  std::vector<tnqe_status> st(n, TNQE_OK);
  if (n == 0) return st;
  std::vector<tnqe_ctx *> ws(W);
  TNQE_HIP(hipEventRecord(ctx->fork_ev, ctx->stream));
  for (int w = 0; w < W; ++w) {
    ws[w] = worker(ctx, w);
    TNQE_HIP(hipStreamWaitEvent(ws[w]->stream, ctx->fork_ev, 0));
  }
  std::atomic<int> next{0};
  auto body = [&](int w) {
    (void)hipSetDevice(ctx->device);
    for (;;) {
      const int q = next.fetch_add(1);
      if (q >= n) return;
      st[order[q]] = run(ws[w], w, order[q]);
    }
  };
  std::vector<std::thread> th;
  for (int w = 1; w < W; ++w) th.emplace_back(body, w);
  body(0);
  for (auto &t : th) t.join();
  return st;
}

}  // namespace

extern "C" {

void tnqe_default_options(tnqe_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->chi = 16;
  o->precision = TNQE_FP64;
  o->eps_S = 1e-12;
  o->tau_w = 1e-13;
  o->max_sweeps = 40;
}

const char *tnqe_version(void) { return "tnqe 0.1 (gfx950)"; }

const char *tnqe_status_string(tnqe_status st) {
  switch (st) {
    case TNQE_OK: return "ok";
    case TNQE_EINVAL: return "invalid argument";
    case TNQE_ESHAPE: return "inconsistent shapes";
    case TNQE_ENOTORTH: return "rotation is not orthogonal";
    case TNQE_EQN: return "tensor breaks particle-number blocks";
    case TNQE_ENOMEM: return "out of memory";
    case TNQE_EWORKSPACE: return "workspace too small";
    case TNQE_EHIP: return "HIP runtime error";
    case TNQE_ESINGULAR: return "overlap matrix singular";
    case TNQE_ENONFINITE: return "non-finite value";
    case TNQE_ENODEVICE: return "no gfx950 device";
  }
  return "unknown status";
}

const char *tnqe_last_error(const tnqe_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

tnqe_status tnqe_create(tnqe_ctx **out, int device, void *stream) {
  if (!out) return TNQE_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= device || device < 0) {
    (void)hipGetLastError();
    return TNQE_ENODEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return TNQE_ENODEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TNQE_ENODEVICE;
  if (hipSetDevice(device) != hipSuccess) return TNQE_EHIP;
  auto *ctx = new tnqe_ctx();
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(stream);
  for (auto &e : ctx->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete ctx;
      return TNQE_EHIP;
    }
  for (auto &e : ctx->svd_ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete ctx;
      return TNQE_EHIP;
    }
  bool ok = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&ctx->sv_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&ctx->sel_ev, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < tnqe_ctx::kAux && ok; ++i)
    ok = hipStreamCreateWithFlags(&ctx->aux[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&ctx->join_ev[i], hipEventDisableTiming) == hipSuccess;
  ok = ok && noalloc_setup(device) == TNQE_OK;
  if (ok) {
    ctx->sv_cap = 1 << 16;
    ok = hipHostMalloc((void **)&ctx->sv_host, ctx->sv_cap * sizeof(double), hipHostMallocDefault) == hipSuccess;
    if (!ok) ctx->sv_cap = 0;
  }
  if (!ok) {
    tnqe_destroy(ctx);
    return TNQE_EHIP;
  }
  *out = ctx;
  return TNQE_OK;
}

tnqe_status tnqe_destroy(tnqe_ctx *ctx) {
  if (!ctx) return TNQE_EINVAL;
  for (tnqe_ctx *w : ctx->sub) tnqe_destroy(w);
  ctx->sub.clear();
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto &e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : ctx->svd_ev)
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < tnqe_ctx::kAux; ++i) {
    if (ctx->aux[i]) (void)hipStreamSynchronize(ctx->aux[i]);
    if (ctx->aux[i]) (void)hipStreamDestroy(ctx->aux[i]);
    if (ctx->join_ev[i]) (void)hipEventDestroy(ctx->join_ev[i]);
  }
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->sv_ev) (void)hipEventDestroy(ctx->sv_ev);
  if (ctx->sel_ev) (void)hipEventDestroy(ctx->sel_ev);
  if (ctx->sv_host) (void)hipHostFree(ctx->sv_host);
  for (auto &e : ctx->env_ev) (void)hipEventDestroy(e);
  if (ctx->own_stream) {
    (void)hipStreamSynchronize(ctx->own_stream);
    (void)hipStreamDestroy(ctx->own_stream);
  }
  delete ctx;
  return TNQE_OK;
}

tnqe_status tnqe_trim(tnqe_ctx *ctx) {
  if (!ctx) return TNQE_EINVAL;
  return guarded(ctx, [&] {
    TNQE_HIP(hipStreamSynchronize(ctx->stream));
    ctx->pool.trim();
  });
}

tnqe_status tnqe_upload(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                        tnqe_problem **out) {
  if (!ctx || !ham || !mps || !out || M < 1) return ctx ? fail(ctx, TNQE_EINVAL, "null argument or M < 1") : TNQE_EINVAL;
  *out = nullptr;
  tnqe_problem *pb = new tnqe_problem();
  tnqe_status st = guarded(ctx, [&] {
    TNQE_HIP(hipSetDevice(ctx->device));
    load_problem(ctx, ham, M, mps, pb);
    place_sites(ctx, pb, mps);
  });
  if (st != TNQE_OK) {
    free_sites(pb);
    delete pb;
    return st;
  }
  *out = pb;
  return TNQE_OK;
}

tnqe_status tnqe_problem_free(tnqe_problem *pb) {
  if (!pb) return TNQE_EINVAL;
  free_sites(pb);
  delete pb;
  return TNQE_OK;
}

namespace {
void copy_out(const SolveOut &so, double *H, double *S, double *E, double *cvec, tnqe_report *rep) {
  std::memcpy(H, so.H.data(), so.H.size() * sizeof(double));
  std::memcpy(S, so.S.data(), so.S.size() * sizeof(double));
  *E = so.E;
  if (cvec) std::memcpy(cvec, so.c.data(), so.c.size() * sizeof(double));
  if (rep) *rep = so.rep;
}
}  // namespace

}  // extern "C"

tnqe_status tnqe::subspace_entry(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                                 const tnqe_options *opts, void *ws, size_t ws_bytes, bool no_alloc,
                                 size_t max_bound, double *H, double *S, double *E, double *c, tnqe_report *rep) {
  if (!ctx || !ham || !mps || !opts || !H || !S || !E) return ctx ? fail(ctx, TNQE_EINVAL, "null argument") : TNQE_EINVAL;
  if (check_options(ctx, opts) != TNQE_OK) return TNQE_EINVAL;
  if (max_bound > 0) {
    // refused before any device work when the bound exceeds the fixed size
    size_t need = 0;
    tnqe_problem pb;
    const tnqe_status st = guarded(ctx, [&] {
      load_problem(ctx, ham, M, mps, &pb);
      need = workspace_bound(ctx, pb, *opts);
    });
    if (st != TNQE_OK) return st;
    if (need > max_bound)
      return fail(ctx, TNQE_EWORKSPACE, "problem needs up to " + std::to_string(need) + " bytes of device memory; " +
                                            "the fixed scratch holds " + std::to_string(max_bound));
  }
  SolveOut so;
  const tnqe_status st = subspace_call(ctx, ham, M, mps, opts, ws, ws_bytes, no_alloc, so);
  if (st != TNQE_OK) return st;
  copy_out(so, H, S, E, c, rep);
  return TNQE_OK;
}

extern "C" {

tnqe_status tnqe_solve(tnqe_ctx *ctx, tnqe_problem *pb, const tnqe_options *opts, double *H, double *S,
                       double *E, double *cvec, tnqe_report *rep) {
  if (!ctx || !pb || !opts || !H || !S || !E) return ctx ? fail(ctx, TNQE_EINVAL, "null argument") : TNQE_EINVAL;
  if (check_options(ctx, opts) != TNQE_OK) return TNQE_EINVAL;
  SolveOut so;
  tnqe_status st = guarded(ctx, [&] {
    TNQE_HIP(hipSetDevice(ctx->device));
    solve_one(ctx, *pb, *opts, so);
    ctx->pool.release_all();
  });
  if (st != TNQE_OK) return st;
  copy_out(so, H, S, E, cvec, rep);
  return TNQE_OK;
}

tnqe_status tnqe_onehot_size(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                             const tnqe_options *opts, int32_t i, int32_t p, int32_t *n) {
  if (!ham || !mps || !opts || !n) return ctx ? fail(ctx, TNQE_EINVAL, "null argument") : TNQE_EINVAL;
  std::unique_ptr<tnqe_ctx> tmp;
  if (!ctx) {
    tmp = std::make_unique<tnqe_ctx>();
    ctx = tmp.get();
  }
  int32_t out = 0;
  tnqe_problem pb;
  const tnqe_status st = guarded(ctx, [&] {
    load_problem(ctx, ham, M, mps, &pb);
    require(i >= 0 && i < M, TNQE_EINVAL, "expanded state out of range");
    require(p >= 0 && p + 1 < pb.N, TNQE_EINVAL, "two-site position out of range");
    out = (int32_t)onehot_list(pb, onehot_dims(pb, i, p), p).size();
  });
  if (st == TNQE_OK) *n = out;
  return st;
}

tnqe_status tnqe_onehot_pencil(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                               const tnqe_options *opts, int32_t i, int32_t p, int32_t n, int32_t *index,
                               double *Hd, double *Sd, double *Hc, double *Sc, tnqe_report *rep) {
  if (!ctx || !ham || !mps || !opts || !index || !Hd || !Sd || !Hc || !Sc)
    return ctx ? fail(ctx, TNQE_EINVAL, "null argument") : TNQE_EINVAL;
  if (check_options(ctx, opts) != TNQE_OK) return TNQE_EINVAL;
  OneHotOut oh;
  tnqe_report r{};
  tnqe_problem pb;
  tnqe_status st = guarded(ctx, [&] {
    TNQE_HIP(hipSetDevice(ctx->device));
    load_problem(ctx, ham, M, mps, &pb);
    place_sites(ctx, &pb, mps);
    onehot_one(ctx, pb, *opts, i, p, oh, r);
    ctx->pool.release_all();
    require((int)oh.index.size() == n, TNQE_ESHAPE,
            "n differs from the number of one-hot entries (" + std::to_string(oh.index.size()) + ")");
  });
  free_sites(&pb);
  if (st != TNQE_OK) return st;
  for (int m = 0; m < n; ++m) {
    index[4 * m] = oh.index[m].x;
    index[4 * m + 1] = oh.index[m].y;
    index[4 * m + 2] = oh.index[m].z;
    index[4 * m + 3] = oh.index[m].w;
  }
  std::memcpy(Hd, oh.Hd.data(), oh.Hd.size() * sizeof(double));
  std::memcpy(Sd, oh.Sd.data(), oh.Sd.size() * sizeof(double));
  std::memcpy(Hc, oh.Hc.data(), oh.Hc.size() * sizeof(double));
  std::memcpy(Sc, oh.Sc.data(), oh.Sc.size() * sizeof(double));
  if (rep) *rep = r;
  return TNQE_OK;
}

tnqe_status tnqe_sweep_step(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                            const tnqe_options *opts, const tnqe_sweep_options *sw, int32_t i, int32_t p,
                            const double *H, const double *S, int32_t *bond_dim, int32_t *bond_qn, int64_t qn_cap,
                            double *sites, int64_t sites_cap, double *U, tnqe_sweep_result *res,
                            tnqe_report *rep) {
  if (!ctx || !ham || !mps || !opts || !sw || !H || !S || !bond_dim || !bond_qn || !sites || !U || !res)
    return ctx ? fail(ctx, TNQE_EINVAL, "null argument") : TNQE_EINVAL;
  if (check_options(ctx, opts) != TNQE_OK) return TNQE_EINVAL;
  SweepOut out;
  tnqe_report r{};
  tnqe_problem pb;
  tnqe_status st = guarded(ctx, [&] {
    TNQE_HIP(hipSetDevice(ctx->device));
    load_problem(ctx, ham, M, mps, &pb);
    require(i >= 0 && i < M, TNQE_EINVAL, "expanded state out of range");
    require(p >= 0 && p + 1 < pb.N, TNQE_EINVAL, "two-site position out of range");
    place_sites(ctx, &pb, mps);
    sweep_one(ctx, pb, *opts, *sw, i, p, H, S, out, r);
    ctx->pool.release_all();
    require((int64_t)out.bond_qn.size() / 2 <= qn_cap, TNQE_ESHAPE,
            "qn_cap too small: " + std::to_string(out.bond_qn.size() / 2) + " labels");
    require((int64_t)out.sites.size() <= sites_cap, TNQE_ESHAPE,
            "sites_cap too small: " + std::to_string(out.sites.size()) + " doubles");
  });
  free_sites(&pb);
  if (st != TNQE_OK) return st;
  std::memcpy(bond_dim, out.bond_dim.data(), out.bond_dim.size() * sizeof(int32_t));
  std::memcpy(bond_qn, out.bond_qn.data(), out.bond_qn.size() * sizeof(int32_t));
  std::memcpy(sites, out.sites.data(), out.sites.size() * sizeof(double));
  std::memcpy(U, out.U.data(), out.U.size() * sizeof(double));
  tnqe_sweep_result q{};
  q.E_old = out.E_old;
  q.E1 = out.E1;
  q.theta = out.theta;
  q.xi_none = out.xi_none;
  q.xi = out.xi;
  q.discarded = out.discarded;
  q.n_onehot = out.n;
  q.n_columns = out.D;
  q.n_kept = out.n_kept;
  q.n_dropped_S = out.n_dropped_S;
  q.accepted = out.accepted;
  q.new_bond = out.new_bond;
  q.E_new = out.E_new;
  q.mit_columns = out.mit_columns;
  q.mit_kept = out.mit_kept;
  *res = q;
  ctx->sweep_t = std::move(out.tnew);
  if (rep) *rep = r;
  return TNQE_OK;
}

tnqe_status tnqe_sweep_last_params(tnqe_ctx *ctx, int32_t n, double *t) {
  if (!ctx || !t) return ctx ? fail(ctx, TNQE_EINVAL, "null argument") : TNQE_EINVAL;
  if (n != (int32_t)ctx->sweep_t.size()) return fail(ctx, TNQE_EINVAL, "n differs from the last sweep step's");
  std::memcpy(t, ctx->sweep_t.data(), ctx->sweep_t.size() * sizeof(double));
  return TNQE_OK;
}

tnqe_status tnqe_solve_batch(tnqe_ctx *ctx, int32_t n, tnqe_problem *const *probs, const tnqe_options *opts,
                             double *const *H, double *const *S, double *E, tnqe_report *rep) {
  if (!ctx || !probs || !opts || !H || !S || !E || n < 0) return ctx ? fail(ctx, TNQE_EINVAL, "null argument") : TNQE_EINVAL;
  for (int s = 0; s < n; ++s) {
    if (!probs[s] || !H[s] || !S[s]) return fail(ctx, TNQE_EINVAL, "null argument");
    if (check_options(ctx, opts + s) != TNQE_OK) return TNQE_EINVAL;
  }
  std::vector<SolveOut> outs(n);
  std::vector<std::string> errs(n);
  std::vector<tnqe_status> st;
  const tnqe_status st0 = guarded(ctx, [&] {
    TNQE_HIP(hipSetDevice(ctx->device));
    std::vector<int> order(n);
    std::vector<double> cost(n);
    for (int s = 0; s < n; ++s) {
      order[s] = s;
      const tnqe_problem &pb = *probs[s];
      const double chi = opts[s].chi_cap_override > 0 ? opts[s].chi_cap_override : opts[s].chi;
      cost[s] = (double)pb.N * pb.N * pb.M * pb.M * chi * chi * chi;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    st = run_batch(ctx, order, batch_workers(n, opts[0]), [&](tnqe_ctx *w, int, int s) {
      const tnqe_status r = guarded(w, [&] {
        TNQE_HIP(hipSetDevice(w->device));
        solve_one(w, *probs[s], opts[s], outs[s]);
        w->pool.release_all();
      });
      if (r != TNQE_OK) errs[s] = w->last_error;
      return r;
    });
  });
  if (st0 != TNQE_OK) return st0;
  for (int s = 0; s < n; ++s)
    if (st[s] != TNQE_OK) return fail(ctx, st[s], "subspace " + std::to_string(s) + ": " + errs[s]);
  for (int s = 0; s < n; ++s) copy_out(outs[s], H[s], S[s], E + s, nullptr, rep ? rep + s : nullptr);
  return TNQE_OK;
}

tnqe_status tnqe_workspace_size(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                                const tnqe_options *opts, size_t *bytes) {
  if (!ham || !mps || !opts || !bytes) return ctx ? fail(ctx, TNQE_EINVAL, "null argument") : TNQE_EINVAL;
  // host-only: without a context a temporary one (no device state) serves
  std::unique_ptr<tnqe_ctx> tmp;
  if (!ctx) {
    tmp = std::make_unique<tnqe_ctx>();
    ctx = tmp.get();
  }
  if (check_options(ctx, opts) != TNQE_OK) return TNQE_EINVAL;
  size_t out = 0;
  tnqe_problem pb;
  tnqe_status st = guarded(ctx, [&] {
    load_problem(ctx, ham, M, mps, &pb);
    out = workspace_bound(ctx, pb, *opts);
  });
  if (st == TNQE_OK) *bytes = out;
  return st;
}

tnqe_status tnqe_subspace(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                          const tnqe_options *opts, void *workspace, size_t ws_bytes, double *H, double *S,
                          double *E, double *c, tnqe_report *rep) {
  return tnqe::subspace_entry(ctx, ham, M, mps, opts, workspace, ws_bytes, false, 0, H, S, E, c, rep);
}

tnqe_status tnqe_subspace_batch(tnqe_ctx *ctx, int32_t n_sub, const tnqe_hamiltonian *ham, const int32_t *M,
                                const tnqe_mps *const *mps, const tnqe_options *opts, void *workspace,
                                size_t ws_bytes, double *const *H, double *const *S, double *E,
                                tnqe_report *rep) {
  if (!ctx || n_sub < 0 || (n_sub > 0 && (!ham || !M || !mps || !opts || !H || !S || !E)))
    return ctx ? fail(ctx, TNQE_EINVAL, "null argument") : TNQE_EINVAL;
  for (int s = 0; s < n_sub; ++s) {
    if (!mps[s] || !H[s] || !S[s]) return fail(ctx, TNQE_EINVAL, "null argument");
    if (check_options(ctx, opts + s) != TNQE_OK) return TNQE_EINVAL;
  }
  std::vector<SolveOut> outs(n_sub);
  std::vector<std::string> errs(n_sub);
  std::vector<tnqe_status> st;
  const tnqe_status st0 = guarded(ctx, [&] {
    TNQE_HIP(hipSetDevice(ctx->device));
    // costs (host-side bounds and estimates) and the worker count: with a
    // workspace, each worker takes an equal part that holds the largest bound
    std::vector<int> order(n_sub);
    std::vector<double> cost(n_sub);
    size_t need = 0;
    for (int s = 0; s < n_sub; ++s) {
      order[s] = s;
      tnqe_problem pb;
      load_problem(ctx, ham + s, M[s], mps[s], &pb);
      const double chi = opts[s].chi_cap_override > 0 ? opts[s].chi_cap_override : opts[s].chi;
      cost[s] = (double)pb.N * pb.N * pb.M * pb.M * chi * chi * chi;
      if (workspace) need = std::max(need, workspace_bound(ctx, pb, opts[s]));
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    int W = batch_workers(n_sub, opts[0]);
    size_t part = 0;
    if (workspace) {
      W = (int)std::max<size_t>(1, std::min<size_t>(W, ws_bytes / std::max<size_t>(need, 1)));
      part = (ws_bytes / W) & ~size_t(255);
    }
    st = run_batch(ctx, order, W, [&](tnqe_ctx *w, int wi, int s) {
      void *ws = workspace ? static_cast<char *>(workspace) + (size_t)wi * part : nullptr;
      const tnqe_status r = subspace_call(w, ham + s, M[s], mps[s], opts + s, ws, workspace ? part : 0, false, outs[s]);
      if (r != TNQE_OK) errs[s] = w->last_error;
      return r;
    });
  });
  if (st0 != TNQE_OK) return st0;
  for (int s = 0; s < n_sub; ++s)
    if (st[s] != TNQE_OK) return fail(ctx, st[s], "subspace " + std::to_string(s) + ": " + errs[s]);
  for (int s = 0; s < n_sub; ++s) copy_out(outs[s], H[s], S[s], E + s, nullptr, rep ? rep + s : nullptr);
  return TNQE_OK;
}

}  // extern "C"

// ============================================================== host-only diagnostics
extern "C" {

tnqe_status tnqe_debug_givens(int32_t N, const double *W, int32_t *pos, double *theta, int32_t *det_sign) {
  if (N < 1 || !W || !pos || !theta || !det_sign) return TNQE_EINVAL;
  std::vector<int> p;
  std::vector<double> t;
  int d = 1;
  givens_plan(N, W, p, t, d);
  for (size_t i = 0; i < p.size(); ++i) {
    pos[i] = p[i];
    theta[i] = t[i];
  }
  *det_sign = d;
  return TNQE_OK;
}

tnqe_status tnqe_debug_host_pool(int32_t workers, int32_t jobs, int64_t *calls) {
  if (workers < 0 || workers > 256 || jobs < 0 || !calls) return TNQE_EINVAL;
  try {
    tnqe::ThreadPool pool(workers);
    std::atomic<int64_t> total{0};
    for (int j = 0; j < jobs; ++j) {
      const int n = 1 + j % 5;
      std::vector<std::atomic<int>> hit(n);
      for (auto &h : hit) h.store(0);
      pool.parallel_for(n, [&](int i) {
        hit[i].fetch_add(1);
        total.fetch_add(1);
      });
      for (auto &h : hit)
        if (h.load() != 1) return TNQE_EINVAL;
    }
    *calls = total.load();
    return TNQE_OK;
  } catch (...) {
    return TNQE_EINVAL;
  }
}

tnqe_status tnqe_debug_select(tnqe_ctx *ctx, int32_t nket, const int32_t *nblk, const int32_t *n,
                              const double *sv, int32_t chi, double tau, int32_t *kept, double *stats) {
  if (!ctx) return TNQE_EINVAL;
  if (nket < 1 || !nblk || !n || !sv || chi < 0 || !(tau >= 0.0) || !kept || !stats)
    return fail(ctx, TNQE_EINVAL, "bad argument to tnqe_debug_select");
  return guarded(ctx, [&] {
    TNQE_HIP(hipSetDevice(ctx->device));
    Call c{ctx};
    const size_t mk = ctx->pool.mark();
    int nbt = 0, maxb = 1, maxv = 0;
    for (int t = 0; t < nket; ++t) {
      require(nblk[t] >= 0, TNQE_EINVAL, "negative block count");
      nbt += nblk[t];
      maxb = std::max(maxb, (int)nblk[t]);
    }
    std::vector<Blk> blks(nbt);
    std::vector<int> kfirst(nket + 1, 0);
    int64_t off = 0;
    for (int t = 0, i = 0; t < nket; ++t) {
      kfirst[t] = i;
      int nv = 0;
      for (int j = 0; j < nblk[t]; ++j, ++i) {
        require(n[i] >= 0, TNQE_EINVAL, "negative value count");
        for (int k = 0; k < n[i]; ++k) {
          const double x = sv[off + k];
          require(std::isfinite(x) && x >= 0.0 && (k == 0 || x <= sv[off + k - 1]), TNQE_EINVAL,
                  "singular values must be finite, non-negative and sorted in decreasing order per block");
        }
        Blk b{};
        b.pair = t;
        b.n = n[i];
        b.sa = j;   // block j of the ket in slot j
        b.sb = 0;
        b.offS = off;
        off += n[i];
        nv += n[i];
        blks[i] = b;
      }
      kfirst[t + 1] = i;
      maxv = std::max(maxv, nv);
    }
    require(select_lds_bytes(maxv, maxb) <= (size_t)kSelectLdsBytes, TNQE_ESHAPE,
            "too many singular values per ket for the truncation kernel");
    KetTables kt{};
    kt.npair = nket;
    kt.N = 1;
    kt.na = maxb - 1;
    kt.nb = 0;
    kt.nslot = maxb;
    kt.btab = c.dev<int2>((size_t)nket * maxb);
    kt.bdim = c.dev<int>(nket);
    const std::vector<double> hsv(sv, sv + off);
    double *dsv = c.upload(hsv);
    Blk *dblk = c.upload(blks);
    const int *dkf = c.upload(kfirst);
    int *dkept = c.dev<int>(std::max(1, nbt));
    double *dstats = c.dev<double>((size_t)3 * nket);
    launch_select(dblk, dkf, nket, maxv, dsv, chi, tau, kt, 0, dkept, dstats, nullptr, ctx->stream);
    c.check_launch();
    std::vector<int> hk(std::max(1, nbt));
    TNQE_HIP(hipMemcpyAsync(hk.data(), dkept, hk.size() * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    TNQE_HIP(hipMemcpyAsync(stats, dstats, (size_t)3 * nket * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    c.sync();
    for (int i = 0; i < nbt; ++i) kept[i] = hk[i];
    ctx->pool.rewind(mk);
  });
}

tnqe_status tnqe_debug_gep(tnqe_ctx *ctx, int32_t M, const double *H, const double *S, double eps_S,
                           double *out) {
  if (!ctx) return TNQE_EINVAL;
  if (M < 1 || M > kMaxM || !H || !S || !out || !(eps_S > 0.0)) return fail(ctx, TNQE_EINVAL, "bad argument to tnqe_debug_gep");
  return guarded(ctx, [&] {
    TNQE_HIP(hipSetDevice(ctx->device));
    Call c{ctx};
    const size_t mk = ctx->pool.mark();
    const std::vector<double> h(H, H + (size_t)M * M), sm(S, S + (size_t)M * M);
    std::vector<int> Ms{M};
    std::vector<int64_t> offs{0};
    double *dout = c.dev<double>(8 + kMaxM);
    launch_gep(c.upload(h), c.upload(sm), c.upload(Ms), c.upload(offs), 1, eps_S, dout, ctx->stream);
    c.check_launch();
    std::vector<double> go(8 + kMaxM);
    TNQE_HIP(hipMemcpyAsync(go.data(), dout, go.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    c.sync();
    std::copy(go.begin(), go.begin() + 8 + M, out);
    ctx->pool.rewind(mk);
  });
}

tnqe_status tnqe_debug_psd_eigen(tnqe_ctx *ctx, int32_t n, const double *A, int32_t path, int32_t max_sweeps,
                                 double *vec, double *val) {
  if (!ctx) return TNQE_EINVAL;
  if (n < 1 || n > 1024 || !A || !vec || !val || path < 0 || path > 4 || max_sweeps < 1)
    return fail(ctx, TNQE_EINVAL, "bad argument to tnqe_debug_psd_eigen");
  return guarded(ctx, [&] {
    TNQE_HIP(hipSetDevice(ctx->device));
    Call c{ctx};
    const size_t mk = ctx->pool.mark();
    const std::vector<double> a(A, A + (size_t)n * n);
    double *dv = nullptr, *dl = nullptr;
    psd_eigen(c, c.upload(a), n, max_sweeps, dv, dl, path);
    TNQE_HIP(hipMemcpyAsync(vec, dv, sizeof(double) * n * n, hipMemcpyDeviceToHost, ctx->stream));
    TNQE_HIP(hipMemcpyAsync(val, dl, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
    c.sync();
    ctx->pool.rewind(mk);
  });
}

tnqe_status tnqe_debug_gate(double theta, double *out) {
  if (!out) return TNQE_EINVAL;
  gate_g4(theta, out);
  return TNQE_OK;
}

tnqe_status tnqe_debug_mpo_dense(int32_t N, const double *h, const double *g, double *Hout, double *Iout,
                                 int32_t *max_bond) {
  if (N < 1 || N > 5 || !h || !g || !Hout || !Iout) return TNQE_EINVAL;
  try {
    MpoStructure m;
    mpo_build_structure(N, m);
    std::vector<double> vals, sv;
    mpo_values(m, h, g, vals, sv);
    // global channel offsets per class
    std::vector<std::vector<int>> base(N + 1);
    std::vector<int> D(N + 1, 0);
    for (int b = 0; b <= N; ++b) {
      for (auto &c : m.classes[b]) {
        base[b].push_back(D[b]);
        D[b] += c.nw;
      }
    }
    int dim = 1;
    std::vector<double> T((size_t)D[0], 1.0);   // bond 0: only I
    for (int x = 0; x < N; ++x) {
      const int nd = dim * 4;
      std::vector<double> Tn((size_t)D[x + 1] * nd * nd, 0.0);
      for (const MpoGroup &grp : m.groups[x]) {
        const OpPattern &P = m.patterns[grp.pattern];
        const double *gv = vals.data() + m.site_nnz_off[x] + grp.val_off;
        auto add = [&](int r, int col, double v) {
          const int wi = base[x][grp.cin] + col, wo = base[x + 1][grp.cout] + r;
          const double *src = T.data() + (size_t)wi * dim * dim;
          double *dst = Tn.data() + (size_t)wo * nd * nd;
          for (int e = 0; e < P.n; ++e)
            for (int i = 0; i < dim; ++i)
              for (int j = 0; j < dim; ++j)
                dst[(size_t)(i * 4 + P.kp[e]) * nd + j * 4 + P.k[e]] += v * P.f[e] * src[(size_t)i * dim + j];
        };
        if (grp.dense) {
          for (int r = 0; r < grp.nr; ++r)
            for (int cc = 0; cc < grp.nc; ++cc) add(grp.r0 + r, grp.c0 + cc, gv[(int64_t)r * grp.nc + cc]);
        } else {
          const int nrow = (int)grp.rowptr.size() - 1;
          for (int r = 0; r < nrow; ++r)
            for (int z = grp.rowptr[r]; z < grp.rowptr[r + 1]; ++z) add(r, grp.col[z], gv[z]);
        }
      }
      T.swap(Tn);
      dim = nd;
    }
    const int wH = base[N][m.final_class] + m.final_H, wI = base[N][m.final_class] + m.final_I;
    std::memcpy(Hout, T.data() + (size_t)wH * dim * dim, sizeof(double) * dim * dim);
    std::memcpy(Iout, T.data() + (size_t)wI * dim * dim, sizeof(double) * dim * dim);
    if (max_bond) *max_bond = m.max_bond;
  } catch (const std::exception &) {
    return TNQE_EINVAL;
  }
  return TNQE_OK;
}

}  // extern "C"
