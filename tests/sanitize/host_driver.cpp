// Host-only checks of libtnqe's C ABI for the sanitizer builds (address and
// undefined behaviour, then thread): the worker pool under back-to-back
// loops, the Givens planner, the MPO builder contracted to dense matrices,
// input validation with its error paths, the workspace bound and the one-hot
// count.  No device is touched (on a machine without a GPU, tnqe_create must
// fail cleanly).  Exits non-zero on any failed check.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tnqe.h"

static int g_fail = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++g_fail;                                                   \
    }                                                             \
  } while (0)

// N x N rotation by angle t on (a, a+1) times a reflection-free mix
static std::vector<double> rotation(int N, double t) {
  std::vector<double> W(N * N, 0.0);
  for (int i = 0; i < N; ++i) W[i * N + i] = 1.0;
  for (int a = 0; a + 1 < N; ++a) {
    const double c = std::cos(t * (a + 1)), s = std::sin(t * (a + 1));
    std::vector<double> R(W);
    for (int r = 0; r < N; ++r) {
      R[r * N + a] = c * W[r * N + a] - s * W[r * N + a + 1];
      R[r * N + a + 1] = s * W[r * N + a] + c * W[r * N + a + 1];
    }
    W = R;
  }
  return W;
}

// a product-state MPS: orbital p occupied by occ[p] (local index k), bond
// dimension 1, labels the running (n_alpha, n_beta)
struct ProductMps {
  std::vector<int32_t> dims, qn;
  std::vector<double> sites, U;
  tnqe_mps m{};
  ProductMps(int N, const std::vector<int> &occ, const std::vector<double> &Ui) : U(Ui) {
    int a = 0, b = 0;
    for (int p = 0; p <= N; ++p) {
      dims.push_back(1);
      qn.push_back(a);
      qn.push_back(b);
      if (p < N) {
        a += occ[p] & 1;
        b += occ[p] >> 1;
      }
    }
    for (int p = 0; p < N; ++p)
      for (int k = 0; k < 4; ++k) sites.push_back(k == occ[p] ? 1.0 : 0.0);
    m.bond_dim = dims.data();
    m.bond_qn = qn.data();
    m.sites = sites.data();
    m.U = U.data();
  }
};

int main() {
  // worker pool: many short loops back to back, several pool sizes
  for (int w : {0, 1, 3, 7, 15}) {
    int64_t calls = 0;
    const int jobs = 4000;
    CHECK(tnqe_debug_host_pool(w, jobs, &calls) == TNQE_OK);
    int64_t want = 0;
    for (int j = 0; j < jobs; ++j) want += 1 + j % 5;
    CHECK(calls == want);
  }
  CHECK(tnqe_debug_host_pool(-1, 10, nullptr) != TNQE_OK);
  // Givens planner on rotations of several sizes
  for (int N : {2, 3, 8, 24}) {
    const std::vector<double> W = rotation(N, 0.37);
    std::vector<int32_t> pos(N * (N - 1) / 2);
    std::vector<double> th(pos.size());
    int32_t det = 0;
    CHECK(tnqe_debug_givens(N, W.data(), pos.data(), th.data(), &det) == TNQE_OK);
    CHECK(det == 1);
  }
  // MPO builder contracted to dense matrices (N <= 5)
  for (int N : {2, 3, 4}) {
    const int D = 1 << (2 * N);
    std::vector<double> h(N * N), g(N * N * N * N), H((size_t)D * D), I((size_t)D * D);
    for (int i = 0; i < N * N; ++i) h[i] = 0.01 * ((i * 7) % 11) - 0.05;
    for (int p = 0; p < N; ++p)
      for (int q = 0; q < N; ++q) h[p * N + q] = h[q * N + p] = 0.5 * (h[p * N + q] + h[q * N + p]);
    for (size_t i = 0; i < g.size(); ++i) g[i] = 0.0;
    for (int p = 0; p < N; ++p) g[((p * N + p) * N + p) * N + p] = 0.3;
    int32_t mb = 0;
    CHECK(tnqe_debug_mpo_dense(N, h.data(), g.data(), H.data(), I.data(), &mb) == TNQE_OK);
    CHECK(mb > 0);
    double asym = 0.0;
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) asym = std::fmax(asym, std::fabs(H[(size_t)i * D + j] - H[(size_t)j * D + i]));
    CHECK(asym < 1e-12);
  }
  // a two-state problem: validation, the workspace bound and the one-hot count
  const int N = 6;
  std::vector<double> hh(N * N, 0.0), L((size_t)N * N * N, 0.0);
  for (int p = 0; p < N; ++p) hh[p * N + p] = -2.0 + 0.4 * p;
  for (int k = 0; k < N; ++k) L[((size_t)k * N + k) * N + k] = 0.2;
  tnqe_hamiltonian ham{N, 3, 3, hh.data(), N, L.data(), nullptr, 0.0};
  std::vector<double> U0(N * N, 0.0);
  for (int p = 0; p < N; ++p) U0[p * N + p] = 1.0;
  ProductMps a(N, {3, 3, 3, 0, 0, 0}, U0), b(N, {3, 1, 2, 3, 0, 0}, rotation(N, 0.21));
  tnqe_mps mps[2] = {a.m, b.m};
  tnqe_options o;
  tnqe_default_options(&o);
  o.chi = 8;
  size_t bytes = 0;
  CHECK(tnqe_workspace_size(nullptr, &ham, 2, mps, &o, &bytes) == TNQE_OK);
  CHECK(bytes > 0);
  int32_t n = 0;
  CHECK(tnqe_onehot_size(nullptr, &ham, 2, mps, &o, 1, 2, &n) == TNQE_OK);
  CHECK(n > 0);
  // error paths: a basis that is not orthogonal, broken labels, bad options
  std::vector<double> Ubad = U0;
  Ubad[0] = 1.01;
  ProductMps c(N, {3, 3, 3, 0, 0, 0}, Ubad);
  tnqe_mps bad[2] = {a.m, c.m};
  CHECK(tnqe_workspace_size(nullptr, &ham, 2, bad, &o, &bytes) == TNQE_ENOTORTH);
  ProductMps d(N, {3, 3, 3, 0, 0, 0}, U0);
  d.qn[2] = 5;
  tnqe_mps badq[2] = {a.m, d.m};
  CHECK(tnqe_workspace_size(nullptr, &ham, 2, badq, &o, &bytes) != TNQE_OK);
  tnqe_options ob = o;
  ob.chi = 0;
  CHECK(tnqe_workspace_size(nullptr, &ham, 2, mps, &ob, &bytes) != TNQE_OK);
  CHECK(tnqe_workspace_size(nullptr, nullptr, 2, mps, &o, &bytes) == TNQE_EINVAL);
  // no device here: creating a context fails cleanly (or succeeds on a GPU machine)
  tnqe_ctx *ctx = nullptr;
  const tnqe_status st = tnqe_create(&ctx, 0, nullptr);
  if (st == TNQE_OK) tnqe_destroy(ctx);
  else CHECK(ctx == nullptr);
  std::printf("host driver: %s (%d failed checks)\n", g_fail ? "FAILED" : "ok", g_fail);
  return g_fail ? 1 : 0;
}
