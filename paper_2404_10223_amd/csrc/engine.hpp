// Host-side state of the library: device memory pool, staging, contexts.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "mpo.hpp"

namespace tnqe {

// Device memory of a call.  By default a grow-only pool of buffers owned by
// the context (hipMalloc on demand, buffers returned to the pool when the call
// ends).  With an arena set, every buffer is carved from that caller-owned
// region instead (a stack: mark/rewind pop what was handed out after the
// mark) and nothing is allocated; running out of it throws TNQE_EWORKSPACE.
class DevicePool {
 public:
  ~DevicePool() { trim(); }
  void *get(size_t bytes);
  void release_all();
  void trim();
  size_t bytes_held() const { return held_; }
  // buffers handed out after mark() go back to the pool at rewind(); safe on a
  // single stream because later work is ordered after earlier work
  size_t mark() const { return order_.size(); }
  void rewind(size_t m);
  // arena mode (base 256-byte aligned); clear_arena() leaves it
  void set_arena(void *base, size_t bytes);
  void clear_arena();
  bool arena() const { return arena_base_ != nullptr; }
  // bytes still available to get() (arena mode), else SIZE_MAX
  size_t available() const;
  size_t arena_peak() const { return arena_peak_; }

 private:
  struct Buf {
    void *p;
    size_t n;
    bool used;
  };
  std::vector<Buf> bufs_;
  std::vector<void *> order_;
  size_t held_ = 0;
  char *arena_base_ = nullptr;
  size_t arena_size_ = 0, arena_top_ = 0, arena_peak_ = 0;
  std::vector<size_t> arena_starts_;   // offset of each handed-out buffer (order_)
};

// Pinned staging area for host-to-device uploads; recycled after each
// stream synchronisation.  With pinned growth disallowed (calls that must not
// allocate through the HIP runtime), space beyond the current pinned buffer
// comes from the host heap (pageable copies, kept until the next reset).
class Staging {
 public:
  ~Staging();
  void *put(const void *src, size_t bytes);   // returns a host copy
  void *reserve(size_t bytes);                // host space to fill
  void reset();
  size_t capacity() const { return cap_; }
  void allow_pinned_growth(bool on) { grow_ = on; }

 private:
  std::vector<std::pair<char *, size_t>> old_;
  std::vector<std::unique_ptr<char[]>> heap_;
  char *buf_ = nullptr;
  size_t cap_ = 0, used_ = 0;
  bool grow_ = true;
};

// Persistent host worker threads for the per-ket loops of the gate phase.
class ThreadPool {
 public:
  explicit ThreadPool(int workers);
  ~ThreadPool();
  // f(i) for i in [0, n) on the workers and the calling thread; returns when
  // all calls are done; the first exception thrown by f is rethrown here
  void parallel_for(int n, const std::function<void(int)> &f);

 private:
  void work(const std::function<void(int)> *f, int n);
  std::vector<std::thread> threads_;
  std::mutex m_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)> *job_ = nullptr;
  int n_ = 0;
  // written under m_; atomic so that waiting threads can poll them briefly
  // before they block on a condition variable
  std::atomic<int> busy_{0};
  std::atomic<unsigned long long> gen_{0};
  std::atomic<bool> stop_{false};
  std::atomic<int> next_{0};
  std::exception_ptr err_;
};

// Row pointers and column indices of every sparse MPO group of one
// structure, on the device (built once per context and site count, or once
// per call inside the caller's workspace, then not owned).
struct MpoDevice {
  int *rowptr = nullptr, *col = nullptr;
  bool owned = true;
  std::vector<std::vector<int64_t>> rp_off, col_off;   // [site][group]
  MpoDevice() = default;
  MpoDevice(const MpoDevice &) = delete;
  MpoDevice &operator=(const MpoDevice &) = delete;
  ~MpoDevice() {
    if (owned && rowptr) (void)hipFree(rowptr);
    if (owned && col) (void)hipFree(col);
  }
};

// One subspace call from host inputs (tnqe_subspace and its variants): with a
// workspace every device buffer lies in it; no_alloc also keeps the call
// from allocating pinned host memory and timing events; max_bound > 0
// refuses, before any device work, problems whose bound exceeds it.
tnqe_status subspace_entry(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                           const tnqe_options *opts, void *ws, size_t ws_bytes, bool no_alloc, size_t max_bound,
                           double *H, double *S, double *E, double *c, tnqe_report *rep);
// The fixed device scratch of the calls that cannot allocate: looked up once
// per device with that device current (defined beside the scratch array).
tnqe_status noalloc_setup(int device);

}  // namespace tnqe

struct tnqe_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  tnqe::DevicePool pool;
  tnqe::Staging staging;
  std::map<int, std::unique_ptr<tnqe::MpoStructure>> mpo_cache;   // by N
  std::map<int, std::unique_ptr<tnqe::MpoDevice>> mpo_dev;        // by N
  std::unique_ptr<tnqe::MpoDevice> mpo_dev_call;                  // in the workspace of this call
  bool no_alloc = false;   // this call must not allocate through the HIP runtime
  hipEvent_t ev[8] = {};
  hipEvent_t svd_ev[128] = {};  // timing of the SVD launches not yet collected
  // pinned host copy of a gate step's kept counts and statistics, and its
  // completion event (created with the context; pageable beyond its size in
  // calls that must not allocate)
  double *sv_host = nullptr;
  size_t sv_cap = 0;
  std::vector<double> sv_pageable;
  hipEvent_t sv_ev = nullptr, sel_ev = nullptr;
  // side streams (default priority) that run independent SVD launches side by
  // side; forked from and joined back into `stream` with events
  static constexpr int kAux = 4;
  hipStream_t aux[kAux] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kAux] = {};
  std::vector<hipEvent_t> env_ev;   // per-launch timing of the environment kernels (grown on demand)
  std::unique_ptr<tnqe::ThreadPool> pool_threads;   // created on first use
  int host_workers = -1;            // threads of pool_threads (-1: one per core, at most 15)
  // tuned tile shapes of the environment GEMMs: (kernel, element bytes, log2
  // of the largest M and N, log2 of the work) -> (tile M, tile N); read from
  // and written to a file on first use of autotuning
  std::map<std::array<int, 5>, std::pair<int, int>> tiles;
  bool tiles_loaded = false;
  std::vector<double> sweep_t;        // parameters t'_m of the last sweep step
  // contexts of the batch workers (same device, each with a stream of its
  // own), created on first use and destroyed with this context
  std::vector<tnqe_ctx *> sub;
  hipStream_t own_stream = nullptr; // a worker's stream (destroyed with it)
};

struct tnqe_problem {
  int N = 0, na = 0, nb = 0, M = 0;
  double e_core = 0.0;
  std::vector<double> h, g;        // reference basis; g = (pq|rs) [N^4]
  std::vector<double> L;           // Cholesky vectors if given [K][N][N]
  int K = 0;
  struct Mps {
    std::vector<int> dims;                   // [N+1]
    std::vector<std::vector<int>> secdim;    // [bond][slot]
    std::vector<double> U;                   // [N][N]
    std::vector<int64_t> site_off;           // [N] offsets into d_sites (doubles)
  };
  std::vector<Mps> mps;
  double *d_sites = nullptr;       // all sites of all MPS
  bool owns_sites = true;          // false: d_sites lies in a call's workspace
  int device = 0;
  int nslot() const { return (na + 1) * (nb + 1); }
};
