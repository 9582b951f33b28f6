// Host-side state of the library: device memory pool, staging, contexts.
#pragma once

#include <hip/hip_runtime.h>

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

// Grow-only pool of device buffers owned by a context.  Buffers handed out
// during a call are returned to the pool when the call ends.
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

 private:
  struct Buf {
    void *p;
    size_t n;
    bool used;
  };
  std::vector<Buf> bufs_;
  std::vector<void *> order_;
  size_t held_ = 0;
};

// Pinned staging area for host-to-device uploads; recycled after each
// stream synchronisation.
class Staging {
 public:
  ~Staging();
  void *put(const void *src, size_t bytes);   // returns pinned copy
  void *reserve(size_t bytes);                // pinned space to fill
  void reset();
  size_t capacity() const { return cap_; }

 private:
  std::vector<std::pair<char *, size_t>> old_;
  char *buf_ = nullptr;
  size_t cap_ = 0, used_ = 0;
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
// structure, on the device (built once per context and site count).
struct MpoDevice {
  int *rowptr = nullptr, *col = nullptr;
  std::vector<std::vector<int64_t>> rp_off, col_off;   // [site][group]
  MpoDevice() = default;
  MpoDevice(const MpoDevice &) = delete;
  MpoDevice &operator=(const MpoDevice &) = delete;
  ~MpoDevice() {
    if (rowptr) (void)hipFree(rowptr);
    if (col) (void)hipFree(col);
  }
};

}  // namespace tnqe

struct tnqe_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  tnqe::DevicePool pool;
  tnqe::Staging staging;
  std::map<int, std::unique_ptr<tnqe::MpoStructure>> mpo_cache;   // by N
  std::map<int, std::unique_ptr<tnqe::MpoDevice>> mpo_dev;        // by N
  hipEvent_t ev[8] = {};
  hipEvent_t svd_ev[128] = {};  // timing of the SVD launches not yet collected
  // pinned host copy of a gate step's singular values, and its completion event
  double *sv_host = nullptr;
  size_t sv_cap = 0;
  hipEvent_t sv_ev = nullptr, sel_ev = nullptr;
  // side streams (default priority) that run independent SVD launches side by
  // side; forked from and joined back into `stream` with events
  static constexpr int kAux = 4;
  hipStream_t aux[kAux] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kAux] = {};
  std::vector<hipEvent_t> env_ev;   // per-launch timing of the environment kernels (grown on demand)
  std::unique_ptr<tnqe::ThreadPool> pool_threads;   // created on first use
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
  int device = 0;
  int nslot() const { return (na + 1) * (nb + 1); }
};
