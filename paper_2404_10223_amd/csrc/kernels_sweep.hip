// Kernels of one generalized-sweep step (Alg. A.1) at a two-site position:
// the expanded pencil in the combined order of eq. subs_exp, the discard of
// linearly dependent columns (App. A2), the whitening of the thresholded
// eigenproblem, the parameter update (eq. param_upd), the rotated two-site
// blocks and their truncation errors (App. A3).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace tnqe {

namespace {

// code[a] >= 0: one-hot state code[a] of the expanded state; code[a] < 0:
// state -code[a] - 1 (unexpanded, its row of the current pencil)
__global__ void k_sw_assemble(const int *code, int D, int n, int M, const double *H, const double *S,
                              const double *Hd, const double *Sd, const double *Hc, const double *Sc, double *Hx,
                              double *Sx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)D * D) return;
  const int a = (int)(e / D), b = (int)(e - (int64_t)a * D);
  const int ca = code[a], cb = code[b];
  double h, s;
  if (ca < 0 && cb < 0) {
    h = H[(int64_t)(-ca - 1) * M + (-cb - 1)];
    s = S[(int64_t)(-ca - 1) * M + (-cb - 1)];
  } else if (ca >= 0 && cb >= 0) {
    h = Hd[(int64_t)ca * n + cb];
    s = Sd[(int64_t)ca * n + cb];
  } else if (ca >= 0) {
    h = Hc[(int64_t)ca * M + (-cb - 1)];
    s = Sc[(int64_t)ca * M + (-cb - 1)];
  } else {
    h = Hc[(int64_t)cb * M + (-ca - 1)];
    s = Sc[(int64_t)cb * M + (-ca - 1)];
  }
  Hx[e] = h;
  Sx[e] = s;
}

// Columns taken in order; column j is kept when its squared distance from the
// span of the kept earlier columns -- the diagonal of the Schur complement
// left by a Cholesky factorisation over the kept columns -- is at least
// tol S_jj.  A (D x D, a copy of S) is overwritten by that factorisation.
// The pivot column goes to LDS once scaled; the trailing update then takes a
// row per wave and consecutive columns per lane (contiguous in A).
constexpr int kDiscardThreads = 1024, kDiscardMaxD = 1024;
__global__ void __launch_bounds__(kDiscardThreads) k_sw_discard(double *A, const double *S, int D, double tol,
                                                                 int *keep) {
  __shared__ double l[kDiscardMaxD];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = kDiscardThreads / 64;
  for (int j = 0; j < D; ++j) {
    __syncthreads();
    const double d = A[(int64_t)j * D + j];
    const bool kj = d > 0.0 && d >= tol * S[(int64_t)j * D + j];
    if (threadIdx.x == 0) keep[j] = kj ? 1 : 0;
    if (!kj) continue;
    const double inv = 1.0 / sqrt(d);
    for (int r = j + 1 + threadIdx.x; r < D; r += kDiscardThreads) {
      const double v = A[(int64_t)r * D + j] * inv;
      A[(int64_t)r * D + j] = v;
      l[r] = v;
    }
    __syncthreads();
    // trailing lower triangle: A[r][c] -= L[r][j] L[c][j], j < c <= r
    for (int r = j + 1 + wave; r < D; r += nwave) {
      const double lr = l[r];
      double *row = A + (int64_t)r * D;
      for (int c = j + 1 + lane; c <= r; c += 64) row[c] -= lr * l[c];
    }
  }
}

__global__ void k_sw_gather(const double *Hx, const double *Sx, int D, const int *kidx, int Dk, double *Hk,
                            double *Sk) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)Dk * Dk) return;
  const int a = (int)(e / Dk), b = (int)(e - (int64_t)a * Dk);
  const int64_t src = (int64_t)kidx[a] * D + kidx[b];
  Hk[e] = Hx[src];
  Sk[e] = Sx[src];
}

// X[row][c] = U_c[row] / sqrt(lam_c), c < r (U: eigenvectors by row, [Dk][Dk])
__global__ void k_sw_whiten(const double *U, const double *lam, int Dk, int r, double *X) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)Dk * r) return;
  const int row = (int)(e / r), c = (int)(e - (int64_t)row * r);
  X[e] = U[(int64_t)c * Dk + row] / sqrt(lam[c]);
}

// B = c I - (C + C^T) / 2 with c = the largest absolute row sum (a bound on
// the largest eigenvalue, so that B is positive semi-definite and its largest
// singular value is c minus the lowest eigenvalue); out[0] = c
constexpr int kShiftThreads = 256;
__global__ void __launch_bounds__(kShiftThreads) k_sw_shift(const double *C, int r, double *B, double *out) {
  __shared__ double part[kShiftThreads];
  double mx = 0.0;
  for (int i = threadIdx.x; i < r; i += kShiftThreads) {
    double s = 0.0;
    for (int j = 0; j < r; ++j) s += fabs(0.5 * (C[(int64_t)i * r + j] + C[(int64_t)j * r + i]));
    mx = fmax(mx, s);
  }
  part[threadIdx.x] = mx;
  __syncthreads();
  for (int o = kShiftThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] = fmax(part[threadIdx.x], part[threadIdx.x + o]);
    __syncthreads();
  }
  const double c = part[0];
  if (threadIdx.x == 0) out[0] = c;
  for (int64_t e = threadIdx.x; e < (int64_t)r * r; e += kShiftThreads) {
    const int i = (int)(e / r), j = (int)(e - (int64_t)i * r);
    B[e] = (i == j ? c : 0.0) - 0.5 * (C[(int64_t)i * r + j] + C[(int64_t)j * r + i]);
  }
}

// t'_m = ck[col[m]] (0 when its column was dropped), normalised, with the sign
// for which sum_m t'_m t_m >= 0 (ties: the largest |t'_m| positive); written
// to tnew and scattered into the dense two-site tensor T (zeroed first)
constexpr int kUpdThreads = 256;
__global__ void __launch_bounds__(kUpdThreads) k_sw_update(const double *ck, const int *col, const double *told,
                                                           int told_ld, int n, const int *dense_of, double *T,
                                                           int64_t tsize, double *tnew, double *stats) {
  __shared__ double s_n[kUpdThreads], s_o[kUpdThreads], s_m[kUpdThreads];
  __shared__ int s_i[kUpdThreads];
  double nn = 0.0, ov = 0.0, am = -1.0;
  int ai = 0;
  for (int m = threadIdx.x; m < n; m += kUpdThreads) {
    const double v = col[m] >= 0 ? ck[col[m]] : 0.0;
    nn += v * v;
    ov += v * told[(int64_t)m * told_ld];
    if (fabs(v) > am) {
      am = fabs(v);
      ai = m;
    }
  }
  s_n[threadIdx.x] = nn;
  s_o[threadIdx.x] = ov;
  s_m[threadIdx.x] = am;
  s_i[threadIdx.x] = ai;
  if (T)
    for (int64_t e = threadIdx.x; e < tsize; e += kUpdThreads) T[e] = 0.0;
  __syncthreads();
  for (int o = kUpdThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s_n[threadIdx.x] += s_n[threadIdx.x + o];
      s_o[threadIdx.x] += s_o[threadIdx.x + o];
      const double m2 = s_m[threadIdx.x + o];
      const int i2 = s_i[threadIdx.x + o];
      if (m2 > s_m[threadIdx.x] || (m2 == s_m[threadIdx.x] && i2 < s_i[threadIdx.x])) {
        s_m[threadIdx.x] = m2;
        s_i[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  const double nrm = sqrt(s_n[0]), o = s_o[0];
  const int im = s_i[0];
  const double vm = col[im] >= 0 ? ck[col[im]] : 0.0;
  const double sg = (o < 0.0 || (o == 0.0 && vm < 0.0)) ? -1.0 : 1.0;
  const double f = nrm > 0.0 ? sg / nrm : 0.0;
  for (int m = threadIdx.x; m < n; m += kUpdThreads) {
    const double v = (col[m] >= 0 ? ck[col[m]] : 0.0) * f;
    tnew[m] = v;
    if (T) T[dense_of[m]] = v;
  }
  if (threadIdx.x == 0) {
    stats[0] = nrm;
    stats[1] = o * f;
  }
}

// One workgroup per block: blk[b].pair = gate index g; rows (k_p segment,
// l), columns (k_{p+1} segment, r); element = sum over (k'_p, k'_{p+1}) of
// G_g[(k_p, k_{p+1}), (k'_p, k'_{p+1})] T[l][k'_p][k'_{p+1}][r].  offp / offq:
// first index of each sector slot in bonds p and p+2.
__global__ void __launch_bounds__(256) k_sw_gate_blocks(const Blk *blk, const double *gates, const double *T,
                                                        int Dq, const int *offp, const int *offq, int na,
                                                        int nb1, double *scratch) {
  const Blk b = blk[blockIdx.x];
  __shared__ double sG[256];
  __shared__ int s_lo[4], s_ro[4];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) sG[i] = gates[(int64_t)b.pair * 256 + i];
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    const int la = b.sa - qk_a(k), lb = b.sb - qk_b(k), ra = b.sa + qk_a(k), rb = b.sb + qk_b(k);
    // (a sector outside the particle numbers has an empty segment)
    s_lo[k] = (la >= 0 && lb >= 0 && la <= na && lb < nb1) ? offp[la * nb1 + lb] : 0;
    s_ro[k] = (ra >= 0 && rb >= 0 && ra <= na && rb < nb1) ? offq[ra * nb1 + rb] : 0;
  }
  __syncthreads();
  double *out = scratch + b.offT;
  for (int64_t e = threadIdx.x; e < (int64_t)b.R * b.C; e += blockDim.x) {
    const int row = (int)(e / b.C), cl = (int)(e - (int64_t)row * b.C);
    int kp = 0, kq = 0;
    while (row >= b.rs[kp + 1]) ++kp;
    while (cl >= b.cs[kq + 1]) ++kq;
    const int l = s_lo[kp] + row - b.rs[kp], r = s_ro[kq] + cl - b.cs[kq];
    const double *g = sG + (kp * 4 + kq) * 16;
    double v = 0.0;
#pragma unroll
    for (int x = 0; x < 16; ++x) v += g[x] * T[(((int64_t)l * 4 + (x >> 2)) * 4 + (x & 3)) * Dq + r];
    out[e] = v;
  }
}

// xi_g = 1 - (sum of the chi largest squared singular values over the blocks
// first[g] .. first[g + 1]); equal values ranked by block order
constexpr int kXiThreads = 256;
__global__ void __launch_bounds__(kXiThreads) k_sw_xi(const Blk *blk, const int *first, const double *scratch,
                                                       int chi, double *xi) {
  extern __shared__ double sv[];
  __shared__ double part[kXiThreads];
  const int g = blockIdx.x, b0 = first[g], b1 = first[g + 1];
  int n = 0;
  for (int b = b0; b < b1; ++b) {
    const Blk &bb = blk[b];
    for (int i = threadIdx.x; i < bb.n; i += kXiThreads) sv[n + i] = scratch[bb.offS + i];
    n += bb.n;
  }
  __syncthreads();
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kXiThreads) {
    const double v = sv[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += (sv[j] > v || (sv[j] == v && j < i)) ? 1 : 0;
    if (rank < chi) s += v * v;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = kXiThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) xi[g] = 1.0 - part[0];
}

// The gate G16 in the one-hot basis: column m (one-hot m = (l, k_p, k_{p+1},
// r)) holds G16[(k_p, k_{p+1}), x] at the one-hot state (l, x, r); one thread
// per column (it also clears the column).  map: dense index -> one-hot index.
__global__ void k_sw_onehot_gate(const int4 *oh, const int *map, int n, int Dq, const double *G16, double *Gm) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  for (int m2 = 0; m2 < n; ++m2) Gm[(int64_t)m2 * n + m] = 0.0;
  const int4 e = oh[m];
  for (int x = 0; x < 16; ++x) {
    const int m2 = map[(((int64_t)e.x * 4 + (x >> 2)) * 4 + (x & 3)) * Dq + e.w];
    if (m2 >= 0) Gm[(int64_t)m2 * n + m] = G16[(e.y * 4 + e.z) * 16 + x];
  }
}

// x[m] = sum_j Ap[l][k_p][j] Aq[j][k_{p+1}][r] at the one-hot entries
__global__ void k_sw_product(const double *Ap, const double *Aq, int Dn, int Dq, const int4 *oh, int n, double *x) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const int4 e = oh[m];
  double v = 0.0;
  for (int j = 0; j < Dn; ++j)
    v += Ap[((int64_t)e.x * 4 + e.y) * Dn + j] * Aq[((int64_t)j * 4 + e.z) * Dq + e.w];
  x[m] = v;
}

// dense tensor T (cleared) with x[m] at dense_of[m]
constexpr int kScatterThreads = 256;
__global__ void __launch_bounds__(kScatterThreads) k_sw_scatter(const double *x, int n, const int *dense_of, double *T,
                                                                 int64_t tsize) {
  for (int64_t e = threadIdx.x; e < tsize; e += kScatterThreads) T[e] = 0.0;
  __syncthreads();
  for (int m = threadIdx.x; m < n; m += kScatterThreads) T[dense_of[m]] = x[m];
}

}  // namespace

void launch_sw_onehot_gate(const int4 *oh, const int *map, int n, int Dq, const double *G16, double *Gm,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_sw_onehot_gate, dim3((n + 127) / 128), dim3(128), 0, st, oh, map, n, Dq, G16, Gm);
}

void launch_sw_product(const double *Ap, const double *Aq, int Dn, int Dq, const int4 *oh, int n, double *x,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_sw_product, dim3((n + 127) / 128), dim3(128), 0, st, Ap, Aq, Dn, Dq, oh, n, x);
}

void launch_sw_scatter(const double *x, int n, const int *dense_of, double *T, int64_t tsize, hipStream_t st) {
  hipLaunchKernelGGL(k_sw_scatter, dim3(1), dim3(kScatterThreads), 0, st, x, n, dense_of, T, tsize);
}

void launch_sw_assemble(const int *code, int D, int n, int M, const double *H, const double *S, const double *Hd,
                        const double *Sd, const double *Hc, const double *Sc, double *Hx, double *Sx,
                        hipStream_t st) {
  const int64_t tot = (int64_t)D * D;
  hipLaunchKernelGGL(k_sw_assemble, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, code, D, n, M, H, S,
                     Hd, Sd, Hc, Sc, Hx, Sx);
}

void launch_sw_discard(double *A, const double *S, int D, double tol, int *keep, hipStream_t st) {
  if (D > kDiscardMaxD) throw Error(TNQE_ESHAPE, "expanded pencil wider than 1024 columns");
  hipLaunchKernelGGL(k_sw_discard, dim3(1), dim3(kDiscardThreads), 0, st, A, S, D, tol, keep);
}

void launch_sw_gather(const double *Hx, const double *Sx, int D, const int *kidx, int Dk, double *Hk, double *Sk,
                      hipStream_t st) {
  const int64_t tot = (int64_t)Dk * Dk;
  hipLaunchKernelGGL(k_sw_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Hx, Sx, D, kidx, Dk, Hk,
                     Sk);
}

void launch_sw_whiten(const double *U, const double *lam, int Dk, int r, double *X, hipStream_t st) {
  const int64_t tot = (int64_t)Dk * r;
  hipLaunchKernelGGL(k_sw_whiten, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, U, lam, Dk, r, X);
}

void launch_sw_shift(const double *C, int r, double *B, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sw_shift, dim3(1), dim3(kShiftThreads), 0, st, C, r, B, out);
}

void launch_sw_update(const double *ck, const int *col, const double *told, int told_ld, int n, const int *dense_of,
                      double *T, int64_t tsize, double *tnew, double *stats, hipStream_t st) {
  hipLaunchKernelGGL(k_sw_update, dim3(1), dim3(kUpdThreads), 0, st, ck, col, told, told_ld, n, dense_of, T, tsize,
                     tnew, stats);
}

void launch_sw_gate_blocks(const Blk *blk, int nblk, const double *gates, const double *T, int Dq, const int *offp,
                           const int *offq, int na, int nb1, double *scratch, hipStream_t st) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_sw_gate_blocks, dim3(nblk), dim3(256), 0, st, blk, gates, T, Dq, offp, offq, na, nb1,
                     scratch);
}

void launch_sw_xi(const Blk *blk, const int *first, int ngate, int max_values, const double *scratch, int chi,
                  double *xi, hipStream_t st) {
  if (ngate == 0) return;
  hipLaunchKernelGGL(k_sw_xi, dim3(ngate), dim3(kXiThreads), (size_t)max_values * sizeof(double), st, blk, first,
                     scratch, chi, xi);
}

}  // namespace tnqe
