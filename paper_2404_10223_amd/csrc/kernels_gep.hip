// M x M generalized eigenproblem H c = E S c on the device in FP64.
//
// S = V diag(lam) V^T by cyclic Jacobi; eigenvalues below eps_S * lam_max are
// dropped; with X = V_kept diag(lam_kept)^(-1/2) the reduced matrix X^T H X is
// diagonalised by Jacobi again; E is its lowest eigenvalue and c = X y.  This
// is the projection form of S thresholding (Sec. V "Regulating the subspace
// condition number", App. A2); kappa_1 = |c|^2 / sqrt(E^2 + 1) (App. A2).
// Sizes are tiny (M <= 32), so one thread per subspace works in LDS.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace tnqe {

namespace {

__device__ void jacobi_eig(double *A, double *V, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * kMaxM + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double a = A[i * kMaxM + j];
        tot += a * a;
        if (i != j) off += a * a;
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * kMaxM + q];
        if (apq == 0.0) continue;
        const double app = A[p * kMaxM + p], aqq = A[q * kMaxM + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {        // A <- A J
          const double akp = A[k * kMaxM + p], akq = A[k * kMaxM + q];
          A[k * kMaxM + p] = c * akp - s * akq;
          A[k * kMaxM + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {        // A <- J^T A
          const double apk = A[p * kMaxM + k], aqk = A[q * kMaxM + k];
          A[p * kMaxM + k] = c * apk - s * aqk;
          A[q * kMaxM + k] = s * apk + c * aqk;
        }
        A[p * kMaxM + q] = A[q * kMaxM + p] = 0.0;
        for (int k = 0; k < n; ++k) {        // V <- V J
          const double vkp = V[k * kMaxM + p], vkq = V[k * kMaxM + q];
          V[k * kMaxM + p] = c * vkp - s * vkq;
          V[k * kMaxM + q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

__global__ void k_gep(const double *H, const double *S, const int *Ms, const int64_t *offs,
                      double eps_S, double *out) {
  __shared__ double A[kMaxM * kMaxM], V[kMaxM * kMaxM], X[kMaxM * kMaxM], W[kMaxM * kMaxM];
  if (threadIdx.x != 0) return;
  const int s = blockIdx.x;
  const int M = Ms[s];
  const double *h = H + offs[s], *sm = S + offs[s];
  double *o = out + (int64_t)s * (8 + kMaxM);
  for (int i = 0; i < 8 + kMaxM; ++i) o[i] = 0.0;
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) A[i * kMaxM + j] = 0.5 * (sm[i * M + j] + sm[j * M + i]);
  jacobi_eig(A, V, M);
  double lmax = -1e300, lmin = 1e300;
  for (int i = 0; i < M; ++i) {
    lmax = fmax(lmax, A[i * kMaxM + i]);
    lmin = fmin(lmin, A[i * kMaxM + i]);
  }
  int nk = 0;
  double lkmin = 1e300;
  for (int i = 0; i < M; ++i) {
    const double l = A[i * kMaxM + i];
    if (l > eps_S * lmax && lmax > 0.0) {
      for (int r = 0; r < M; ++r) X[r * kMaxM + nk] = V[r * kMaxM + i] / sqrt(l);
      lkmin = fmin(lkmin, l);
      ++nk;
    }
  }
  o[3] = (double)(M - nk);
  o[2] = lmin;
  if (nk == 0) {
    o[5] = 1.0;   // singular
    return;
  }
  o[1] = lmax / lkmin;
  // W = H X  [M x nk], A = X^T W  [nk x nk]
  for (int r = 0; r < M; ++r)
    for (int j = 0; j < nk; ++j) {
      double acc = 0.0;
      for (int k = 0; k < M; ++k) acc += 0.5 * (h[r * M + k] + h[k * M + r]) * X[k * kMaxM + j];
      W[r * kMaxM + j] = acc;
    }
  for (int i = 0; i < nk; ++i)
    for (int j = 0; j < nk; ++j) {
      double acc = 0.0;
      for (int k = 0; k < M; ++k) acc += X[k * kMaxM + i] * W[k * kMaxM + j];
      A[i * kMaxM + j] = acc;
    }
  for (int i = 0; i < nk; ++i)
    for (int j = i + 1; j < nk; ++j) {
      const double a = 0.5 * (A[i * kMaxM + j] + A[j * kMaxM + i]);
      A[i * kMaxM + j] = A[j * kMaxM + i] = a;
    }
  jacobi_eig(A, V, nk);
  int i0 = 0;
  for (int i = 1; i < nk; ++i)
    if (A[i * kMaxM + i] < A[i0 * kMaxM + i0]) i0 = i;
  const double E = A[i0 * kMaxM + i0];
  double cc = 0.0;
  for (int r = 0; r < M; ++r) {
    double acc = 0.0;
    for (int k = 0; k < nk; ++k) acc += X[r * kMaxM + k] * V[k * kMaxM + i0];
    o[8 + r] = acc;
    cc += acc * acc;
  }
  o[0] = E;
  o[4] = cc / sqrt(E * E + 1.0);
}

}  // namespace

void launch_gep(const double *H, const double *S, const int *Ms, const int64_t *offs, int nsub,
                double eps_S, double *out, hipStream_t st) {
  if (nsub == 0) return;
  hipLaunchKernelGGL(k_gep, dim3(nsub), dim3(64), 0, st, H, S, Ms, offs, eps_S, out);
}

}  // namespace tnqe
