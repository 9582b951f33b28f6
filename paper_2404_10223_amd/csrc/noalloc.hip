// tnqe_subspace_noalloc: tnqe_subspace for callers that cannot allocate
// memory (code under stream capture, tight serving loops, harnesses that
// forbid allocation).  Its device memory is one fixed array per GPU, held
// from the first context on that GPU until the process ends.
#include "engine.hpp"

#include <mutex>

namespace {

// Largest device footprint of a no-alloc call (the workspace bound of its
// inputs must not exceed it).
constexpr size_t kNoAllocBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;

// The scratch: one copy per GPU at its own address.  Host code never uses
// the array's name as an address: it uses the per-device pointer that
// hipGetSymbolAddress returned for that device.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

// Once per device, with that device current (called by tnqe_create).
tnqe_status tnqe::noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return TNQE_ENODEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return TNQE_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return TNQE_EHIP;
  }
  g_ptr[device] = p;
  return TNQE_OK;
}

extern "C" {

size_t tnqe_noalloc_capacity(void) { return kNoAllocBytes; }

tnqe_status tnqe_subspace_noalloc(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                                  const tnqe_options *opts, double *H, double *S, double *E, double *c,
                                  tnqe_report *rep) {
  if (!ctx) return TNQE_EINVAL;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_ptr[ctx->device];
  }
  if (!base) {
    ctx->last_error = "no scratch address for this device (context not created by tnqe_create)";
    return TNQE_EHIP;
  }
  return tnqe::subspace_entry(ctx, ham, M, mps, opts, base, kNoAllocBytes, true, kNoAllocBytes, H, S, E, c, rep);
}

}  // extern "C"
