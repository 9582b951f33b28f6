// Gate phase on gfx950: two-site gate contraction, split of the truncated
// factors, and exact centre moves (the SVDs are in kernels_svd.hip).
//
// Every kernel works on a list of quantum-number blocks (one workgroup per
// block).  Blocks of all kets in flight are launched together, so one launch
// covers every pair of the subspace at the same gate position.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace tnqe {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ inline int seg_of(const int *s, int x) {
  int k = 0;
  while (k < 3 && x >= s[k + 1]) ++k;
  return k;
}

// T'[row, col] = sum_{k1,k2} G[(k1',k2'),(k1,k2)] sum_m A_a[l,k1,m] A_{a+1}[m,k2,r]
__global__ void __launch_bounds__(kThreads) k_two_site(KetTables kt, int a, const Blk *blks,
                                                       const double *gates, double *scratch) {
  const Blk b = blks[blockIdx.x];
  const int pair = b.pair;
  const double *A = kt.site[pair * kt.N + a];
  const double *B = kt.site[pair * kt.N + a + 1];
  const int Dm = kt.dim(a + 1, pair), Dr = kt.dim(a + 2, pair);
  const double *G = gates + (int64_t)pair * 256;
  double *T = scratch + b.offT;
  __shared__ double sG[256];
  for (int i = threadIdx.x; i < 256; i += kThreads) sG[i] = G[i];
  __syncthreads();
  const int total = b.R * b.C;
  for (int idx = threadIdx.x; idx < total; idx += kThreads) {
    const int row = idx / b.C, col = idx - row * b.C;
    const int k1p = seg_of(b.rs, row), k2p = seg_of(b.cs, col);
    const int la = b.sa - qk_a(k1p), lb = b.sb - qk_b(k1p);
    const int ra = b.sa + qk_a(k2p), rb = b.sb + qk_b(k2p);
    const int l = kt.sec(a, pair, la, lb).x + (row - b.rs[k1p]);
    const int r = kt.sec(a + 2, pair, ra, rb).x + (col - b.cs[k2p]);
    double acc = 0.0;
    for (int k1 = 0; k1 < 4; ++k1) {
      const int2 mid = kt.sec(a + 1, pair, la + qk_a(k1), lb + qk_b(k1));
      if (mid.y == 0) continue;
      const double *arow = A + ((int64_t)l * 4 + k1) * Dm + mid.x;
      for (int k2 = 0; k2 < 4; ++k2) {
        const double g = sG[(k1p * 4 + k2p) * 16 + k1 * 4 + k2];
        if (g == 0.0) continue;
        const double *bcol = B + ((int64_t)mid.x * 4 + k2) * Dr + r;
        double s = 0.0;
        for (int m = 0; m < mid.y; ++m) s += arow[m] * bcol[(int64_t)m * 4 * Dr];
        acc += g * s;
      }
    }
    T[idx] = acc;
  }
}

// New A_a columns and A_{a+1} rows of one kept block (zero, then scatter).
__global__ void __launch_bounds__(kThreads) k_split_gate(KetTables kt, int a, const Blk *blks,
                                                         const double *scratch) {
  const Blk b = blks[blockIdx.x];
  if (b.kept == 0) return;
  const int pair = b.pair;
  double *A = kt.site[pair * kt.N + a];
  double *B = kt.site[pair * kt.N + a + 1];
  const int Dl = kt.dim(a, pair), Dn = kt.dim(a + 1, pair), Dr = kt.dim(a + 2, pair);
  const double *U = scratch + b.offU, *Bo = scratch + b.offB;
  const int kept = b.kept;
  for (int64_t e = threadIdx.x; e < (int64_t)Dl * 4 * kept; e += kThreads) {
    const int64_t row = e / kept;
    A[row * Dn + b.j0 + (e - row * kept)] = 0.0;
  }
  for (int64_t e = threadIdx.x; e < (int64_t)kept * 4 * Dr; e += kThreads)
    B[(int64_t)b.j0 * 4 * Dr + e] = 0.0;
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)b.R * kept; e += kThreads) {
    const int row = e / kept, jj = e - (int64_t)row * kept;
    const int k = seg_of(b.rs, row);
    const int l = kt.sec(a, pair, b.sa - qk_a(k), b.sb - qk_b(k)).x + (row - b.rs[k]);
    A[((int64_t)l * 4 + k) * Dn + b.j0 + jj] = U[(int64_t)jj * b.R + row];
  }
  for (int64_t e = threadIdx.x; e < (int64_t)kept * b.C; e += kThreads) {
    const int jj = e / b.C, col = e - (int64_t)jj * b.C;
    const int k = seg_of(b.cs, col);
    const int r = kt.sec(a + 2, pair, b.sa + qk_a(k), b.sb + qk_b(k)).x + (col - b.cs[k]);
    B[((int64_t)(b.j0 + jj) * 4 + k) * Dr + r] = Bo[(int64_t)jj * b.C + col];
  }
}

// LQ move at site q: block = rows of sector s of bond q, columns (k, r).
// aux0 = offset of the sector in the (old) bond q.
__global__ void __launch_bounds__(kThreads) k_gather_lq(KetTables kt, int q, const Blk *blks,
                                                        double *scratch) {
  const Blk b = blks[blockIdx.x];
  const int pair = b.pair;
  const double *A = kt.site[pair * kt.N + q];
  const int Dr = kt.dim(q + 1, pair);
  double *T = scratch + b.offT;
  for (int64_t e = threadIdx.x; e < (int64_t)b.R * b.C; e += kThreads) {
    const int row = e / b.C, col = e - (int64_t)row * b.C;
    const int k = seg_of(b.cs, col);
    const int r = kt.sec(q + 1, pair, b.sa + qk_a(k), b.sb + qk_b(k)).x + (col - b.cs[k]);
    T[e] = A[((int64_t)(b.aux0 + row) * 4 + k) * Dr + r];
  }
}

// A_q rows <- V^T rows; A_{q-1} columns <- old A_{q-1} U Sigma.
// aux0 = old offset of the sector in bond q, aux1 = old dimension of bond q.
__global__ void __launch_bounds__(kThreads) k_apply_lq(KetTables kt, int q, const Blk *blks,
                                                       const double *scratch,
                                                       double *const *old_left) {
  const Blk b = blks[blockIdx.x];
  const int pair = b.pair;
  double *A = kt.site[pair * kt.N + q];
  double *P = kt.site[pair * kt.N + q - 1];
  const double *Po = old_left[pair];
  const int Dr = kt.dim(q + 1, pair), Dn = kt.dim(q, pair), Dl = kt.dim(q - 1, pair);
  const int Dold = b.aux1, n = b.n;
  const double *U = scratch + b.offU, *Bo = scratch + b.offB, *S = scratch + b.offS;
  for (int64_t e = threadIdx.x; e < (int64_t)n * 4 * Dr; e += kThreads) A[(int64_t)b.j0 * 4 * Dr + e] = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)Dl * 4 * n; e += kThreads) {
    const int64_t row = e / n;
    P[row * Dn + b.j0 + (e - row * n)] = 0.0;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)n * b.C; e += kThreads) {
    const int jj = e / b.C, col = e - (int64_t)jj * b.C;
    const int k = seg_of(b.cs, col);
    const int r = kt.sec(q + 1, pair, b.sa + qk_a(k), b.sb + qk_b(k)).x + (col - b.cs[k]);
    const double s = S[jj];
    A[((int64_t)(b.j0 + jj) * 4 + k) * Dr + r] = s > 0.0 ? Bo[(int64_t)jj * b.C + col] / s : 0.0;
  }
  for (int k = 0; k < 4; ++k) {
    const int2 ls = kt.sec(q - 1, pair, b.sa - qk_a(k), b.sb - qk_b(k));
    for (int64_t e = threadIdx.x; e < (int64_t)ls.y * n; e += kThreads) {
      const int li = e / n, jj = e - (int64_t)li * n;
      const double *prow = Po + ((int64_t)(ls.x + li) * 4 + k) * Dold + b.aux0;
      double acc = 0.0;
      const double *ucol = U + (int64_t)jj * b.R;
      for (int mm = 0; mm < b.R; ++mm) acc += prow[mm] * ucol[mm];
      P[((int64_t)(ls.x + li) * 4 + k) * Dn + b.j0 + jj] = acc * S[jj];
    }
  }
}

// QR move at site p: block = rows (k, l) feeding sector s of bond p+1, columns r in s.
// aux0 = offset of the sector in the (old) bond p+1.
__global__ void __launch_bounds__(kThreads) k_gather_qr(KetTables kt, int p, const Blk *blks,
                                                        double *scratch) {
  const Blk b = blks[blockIdx.x];
  const int pair = b.pair;
  const double *A = kt.site[pair * kt.N + p];
  const int Dr = kt.dim(p + 1, pair);
  double *T = scratch + b.offT;
  for (int64_t e = threadIdx.x; e < (int64_t)b.R * b.C; e += kThreads) {
    const int row = e / b.C, col = e - (int64_t)row * b.C;
    const int k = seg_of(b.rs, row);
    const int l = kt.sec(p, pair, b.sa - qk_a(k), b.sb - qk_b(k)).x + (row - b.rs[k]);
    T[e] = A[((int64_t)l * 4 + k) * Dr + b.aux0 + col];
  }
}

// A_p columns <- U; A_{p+1} rows <- B (old A_{p+1}).
// aux0 = old offset of the sector in bond p+1, aux1 = old dimension of bond p+1.
__global__ void __launch_bounds__(kThreads) k_apply_qr(KetTables kt, int p, const Blk *blks,
                                                       const double *scratch,
                                                       double *const *old_right) {
  const Blk b = blks[blockIdx.x];
  const int pair = b.pair;
  double *A = kt.site[pair * kt.N + p];
  double *Nx = kt.site[pair * kt.N + p + 1];
  const double *No = old_right[pair];
  const int Dn = kt.dim(p + 1, pair), Dl = kt.dim(p, pair), Drr = kt.dim(p + 2, pair);
  const int n = b.n;
  const double *U = scratch + b.offU, *Bo = scratch + b.offB;
  for (int64_t e = threadIdx.x; e < (int64_t)Dl * 4 * n; e += kThreads) {
    const int64_t row = e / n;
    A[row * Dn + b.j0 + (e - row * n)] = 0.0;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)b.R * n; e += kThreads) {
    const int row = e / n, jj = e - (int64_t)row * n;
    const int k = seg_of(b.rs, row);
    const int l = kt.sec(p, pair, b.sa - qk_a(k), b.sb - qk_b(k)).x + (row - b.rs[k]);
    A[((int64_t)l * 4 + k) * Dn + b.j0 + jj] = U[(int64_t)jj * b.R + row];
  }
  const int W = 4 * Drr;
  for (int64_t e = threadIdx.x; e < (int64_t)n * W; e += kThreads) {
    const int jj = e / W, x = e - (int64_t)jj * W;
    double acc = 0.0;
    for (int mm = 0; mm < b.C; ++mm) acc += Bo[(int64_t)jj * b.C + mm] * No[(int64_t)(b.aux0 + mm) * W + x];
    Nx[(int64_t)(b.j0 + jj) * W + x] = acc;
  }
}

__global__ void k_copy(double *const *dst, double *const *src, const int64_t *count) {
  const int i = blockIdx.y;
  const int64_t n = count[i];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[i][e] = src[i][e];
}

__global__ void k_site_sign(double *const *site, const int *rows, int cols) {
  const int i = blockIdx.y;
  const int64_t n = (int64_t)rows[i] * 4 * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (e / cols) % 4;
    if (k == 1 || k == 2) site[i][e] = -site[i][e];
  }
}

}  // namespace

void launch_two_site(const KetTables &kt, int a, const Blk *blk, int nblk, const double *gates,
                     double *scratch, hipStream_t st) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_two_site, dim3(nblk), dim3(kThreads), 0, st, kt, a, blk, gates, scratch);
}

void launch_split_gate(const KetTables &kt, int a, const Blk *blk, int nblk, const double *scratch,
                       hipStream_t st) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_split_gate, dim3(nblk), dim3(kThreads), 0, st, kt, a, blk, scratch);
}

void launch_gather_lq(const KetTables &kt, int q, const Blk *blk, int nblk, double *scratch,
                      hipStream_t st) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_gather_lq, dim3(nblk), dim3(kThreads), 0, st, kt, q, blk, scratch);
}

void launch_apply_lq(const KetTables &kt, int q, const Blk *blk, int nblk, const double *scratch,
                     double *const *old_left, hipStream_t st) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_apply_lq, dim3(nblk), dim3(kThreads), 0, st, kt, q, blk, scratch, old_left);
}

void launch_gather_qr(const KetTables &kt, int p, const Blk *blk, int nblk, double *scratch,
                      hipStream_t st) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_gather_qr, dim3(nblk), dim3(kThreads), 0, st, kt, p, blk, scratch);
}

void launch_apply_qr(const KetTables &kt, int p, const Blk *blk, int nblk, const double *scratch,
                     double *const *old_right, hipStream_t st) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_apply_qr, dim3(nblk), dim3(kThreads), 0, st, kt, p, blk, scratch, old_right);
}

void launch_copy(double *const *dst, double *const *src, const int64_t *count, int n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_copy, dim3(64, n), dim3(256), 0, st, dst, src, count);
}

void launch_site_sign(double *const *site, const int *rows, int n, int cols, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_site_sign, dim3(16, n), dim3(256), 0, st, site, rows, cols);
}

}  // namespace tnqe
