// Environment sweep on gfx950: re-layout of site tensors into a common
// sector-padded layout, grouped block GEMMs (bra^T x Y and L x ket), the
// channel mix with the MPO, and the compensated final element.
//
// Environment layout at bond b, per MPO channel class c (shift d = bra sector -
// ket sector) and ket sector s: a dense block [dim_bra(s + d)][n_channels(c)]
// [dim_ket(s)] ("bra-major"), so both contractions of a site are plain GEMMs
// whose long dimension runs over (bra index, channel) or (channel, ket index).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace tnqe {

namespace {

// ------------------------------------------------------------------ GEMM
// One workgroup computes a TM x TN tile of C for one problem and one pair.
// Each of the 256 threads owns an RM x RN micro-tile; K is staged through LDS
// in chunks of KC.
template <typename T, int TM, int TN, int RM, int RN>
__global__ void __launch_bounds__(256) k_bgemm(const GemmDesc *descs, int ndesc, PairPtrs pp) {
  constexpr int KC = 16;
  constexpr int TX = TN / RN;   // threads along N
  static_assert((TM / RM) * (TN / RN) == 256, "tile");
  __shared__ T sA[KC][TM + 1];
  __shared__ T sB[KC][TN];
  const int pair = blockIdx.y;
  // locate the problem owning this tile
  int lo = 0, hi = ndesc - 1;
  const int tile = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  const GemmDesc &d = descs[lo];
  const int per = d.tilesM * d.tilesN;
  const int t0 = tile - d.tile0;
  const int bt = t0 / per, t = t0 - bt * per;
  const int m0 = (t / d.tilesN) * TM, n0 = (t % d.tilesN) * TN;
  const T *Abase = static_cast<const T *>(pp.A[pair]) + bt * d.sA;
  const T *Bbase = static_cast<const T *>(pp.B[pair]) + bt * d.sB;
  T *Cb = static_cast<T *>(pp.C[pair]) + d.offC + bt * d.sC;
  const T alpha = (T)d.alpha;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  T acc[RM][RN];
#pragma unroll
  for (int i = 0; i < RM; ++i)
#pragma unroll
    for (int j = 0; j < RN; ++j) acc[i][j] = T(0);
  for (int sgi = 0; sgi < d.nseg; ++sgi) {
    const GemmSeg sg = d.seg[sgi];
    const T *A = Abase + sg.offA;
    const T *B = Bbase + sg.offB;
    for (int k0 = 0; k0 < sg.K; k0 += KC) {
      for (int e = threadIdx.x; e < KC * TM; e += 256) {
        int kk, mm;
        if (sg.transA) { mm = e % TM; kk = e / TM; } else { kk = e % KC; mm = e / KC; }
        const int gm = m0 + mm, gk = k0 + kk;
        T v = T(0);
        if (gm < d.M && gk < sg.K)
          v = sg.transA ? A[(int64_t)gk * sg.lda + gm] : A[(int64_t)gm * sg.lda + gk];
        sA[kk][mm] = v;
      }
      for (int e = threadIdx.x; e < KC * TN; e += 256) {
        const int kk = e / TN, nn = e % TN;
        const int gn = n0 + nn, gk = k0 + kk;
        sB[kk][nn] = (gn < d.N && gk < sg.K) ? B[(int64_t)gk * sg.ldb + gn] : T(0);
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        T a[RM], b[RN];
#pragma unroll
        for (int i = 0; i < RM; ++i) a[i] = sA[kk][ty * RM + i];
#pragma unroll
        for (int j = 0; j < RN; ++j) b[j] = sB[kk][tx + j * TX];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
          for (int j = 0; j < RN; ++j) acc[i][j] += a[i] * b[j];
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    const int gm = m0 + ty * RM + i;
    if (gm >= d.M) continue;
#pragma unroll
    for (int j = 0; j < RN; ++j) {
      const int gn = n0 + tx + j * TX;
      if (gn < d.N) {
        T *c = Cb + (int64_t)gm * d.ldc + gn;
        *c = d.beta ? *c + alpha * acc[i][j] : alpha * acc[i][j];
      }
    }
  }
}

// ------------------------------------------------------------------ channel mix
template <typename T>
__global__ void __launch_bounds__(256) k_mix(MixArgs a, const T *const *X, T *const *Y) {
  const int pair = blockIdx.y;
  int lo = 0, hi = a.ntask - 1;
  const int chunk = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.task_chunk0[mid] <= chunk) lo = mid; else hi = mid - 1;
  }
  const MixTask tk = a.tasks[lo];
  const int64_t e = (int64_t)(chunk - a.task_chunk0[lo]) * 256 + threadIdx.x;
  const int64_t total = (int64_t)tk.da * tk.nw_out * tk.db;
  if (e >= total) return;
  const int b = e % tk.db;
  const int w = (e / tk.db) % tk.nw_out;
  const int ap = e / ((int64_t)tk.db * tk.nw_out);
  const double *vals = a.vals + a.basis[pair] * a.basis_stride + a.site_off;
  const T *Xp = X[pair];
  double acc = 0.0;
  for (int si = 0; si < tk.nsrc; ++si) {
    const MixSrc s = a.src[tk.src0 + si];
    const CsrGroup g = a.groups[s.group];
    const int r0 = a.rowptr[g.rowptr + w], r1 = a.rowptr[g.rowptr + w + 1];
    const T *xb = Xp + s.offX + ((int64_t)ap * s.nw_in) * tk.db + b;
    double part = 0.0;
    for (int z = r0; z < r1; ++z) part += vals[g.val + z] * (double)xb[(int64_t)a.col[g.col + z] * tk.db];
    acc += s.factor * part;
  }
  Y[pair][tk.offY + e] = (T)acc;
}

template <typename T>
__global__ void k_env_init(T *const *L, int64_t size) {
  T *p = L[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < size; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = (e == 0) ? T(1) : T(0);
}

// error-free transformation: s + e = a + b exactly
__device__ inline void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// last site: out[pair * nw + w] = sum_{k', a'} bra[a', k', 0] Y_k'[a'][w][0]
template <typename T>
__global__ void __launch_bounds__(256) k_env_final(const double *const *bra, const T *const *Y,
                                                   const int64_t *offY, const int *da,
                                                   const int64_t *offBra, int nw, int nk,
                                                   double *out) {
  const int pair = blockIdx.x;
  __shared__ double ss[256], se[256];
  for (int w = 0; w < nw; ++w) {
    double s = 0.0, c = 0.0;
    for (int k = 0; k < nk; ++k) {
      const T *y = Y[pair] + offY[k];
      const double *bp = bra[pair] + offBra[k];
      for (int i = threadIdx.x; i < da[k]; i += 256) {
        // bra index i of the sector, local state k: bra[(off + i) * 4 + k]
        const double p = bp[(int64_t)i * 4] * (double)y[(int64_t)i * nw + w];
        double t, e;
        two_sum(s, p, t, e);
        s = t;
        c += e;
      }
    }
    ss[threadIdx.x] = s;
    se[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) {
        double t, e;
        two_sum(ss[threadIdx.x], ss[threadIdx.x + o], t, e);
        ss[threadIdx.x] = t;
        se[threadIdx.x] += se[threadIdx.x + o] + e;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)pair * nw + w] = ss[0] + se[0];
    __syncthreads();
  }
}

// padded re-layout of one site for many MPS: dst[lp][k][rp] from src[l][k][r]
template <typename T>
__global__ void k_repack(const double *const *src, T *const *dst, const int2 *srcl, const int2 *srcr,
                         const int *srcDr, int nslot, const int2 *pmapl, const int2 *pmapr, int Dpl,
                         int Dpr) {
  const int it = blockIdx.y;
  const int64_t total = (int64_t)Dpl * 4 * Dpr;
  const double *S = src[it];
  T *D = dst[it];
  const int2 *tl = srcl + (int64_t)it * nslot, *tr = srcr + (int64_t)it * nslot;
  const int Dr = srcDr[it];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int rp = e % Dpr;
    const int k = (e / Dpr) % 4;
    const int lp = e / (4 * (int64_t)Dpr);
    const int2 ml = pmapl[lp], mr = pmapr[rp];     // (slot, index within sector)
    const int2 sl = tl[ml.x], sr = tr[mr.x];       // (offset, dim) in the source
    T v = T(0);
    if (ml.y < sl.y && mr.y < sr.y) v = (T)S[((int64_t)(sl.x + ml.y) * 4 + k) * Dr + sr.x + mr.y];
    D[e] = v;
  }
}

}  // namespace

template <typename T>
void launch_bgemm(const GemmDesc *d, int ndesc, int ntiles, int tileM, int tileN, PairPtrs pp,
                  int npair, hipStream_t st) {
  if (ndesc == 0 || ntiles == 0 || npair == 0) return;
  dim3 grid(ntiles, npair);
  if (tileM == 256 && tileN == 16)
    hipLaunchKernelGGL((k_bgemm<T, 256, 16, 16, 1>), grid, dim3(256), 0, st, d, ndesc, pp);
  else if (tileM == 16 && tileN == 256)
    hipLaunchKernelGGL((k_bgemm<T, 16, 256, 1, 16>), grid, dim3(256), 0, st, d, ndesc, pp);
  else if (tileM == 128 && tileN == 32)
    hipLaunchKernelGGL((k_bgemm<T, 128, 32, 8, 2>), grid, dim3(256), 0, st, d, ndesc, pp);
  else if (tileM == 32 && tileN == 128)
    hipLaunchKernelGGL((k_bgemm<T, 32, 128, 2, 8>), grid, dim3(256), 0, st, d, ndesc, pp);
  else
    hipLaunchKernelGGL((k_bgemm<T, 64, 64, 4, 4>), grid, dim3(256), 0, st, d, ndesc, pp);
}

template <typename T>
void launch_mix(const MixArgs &a, const T *const *X, T *const *Y, int npair, hipStream_t st) {
  if (a.ntask == 0 || a.nchunk == 0 || npair == 0) return;
  hipLaunchKernelGGL(k_mix<T>, dim3(a.nchunk, npair), dim3(256), 0, st, a, X, Y);
}

template <typename T>
void launch_env_init(T *const *L, int npair, int64_t size, hipStream_t st) {
  if (npair == 0) return;
  hipLaunchKernelGGL(k_env_init<T>, dim3(1, npair), dim3(64), 0, st, L, size);
}

template <typename T>
void launch_env_final(const double *const *bra, const T *const *Y, const int64_t *offY,
                      const int *da, const int64_t *offBra, int nw, int nk, double *out,
                      int npair, hipStream_t st) {
  if (npair == 0) return;
  hipLaunchKernelGGL(k_env_final<T>, dim3(npair), dim3(256), 0, st, bra, Y, offY, da, offBra, nw, nk, out);
}

template <typename T>
void launch_repack(const double *const *src, T *const *dst, const int2 *srcl, const int2 *srcr,
                   const int *srcDr, int nslot, const int2 *pmapl, const int2 *pmapr, int Dpl, int Dpr,
                   int nitem, hipStream_t st) {
  if (nitem == 0) return;
  const int64_t total = (int64_t)Dpl * 4 * Dpr;
  int bx = (int)((total + 255) / 256);
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_repack<T>, dim3(bx, nitem), dim3(256), 0, st, src, dst, srcl, srcr, srcDr, nslot,
                     pmapl, pmapr, Dpl, Dpr);
}

template void launch_bgemm<double>(const GemmDesc *, int, int, int, int, PairPtrs, int, hipStream_t);
template void launch_bgemm<float>(const GemmDesc *, int, int, int, int, PairPtrs, int, hipStream_t);
template void launch_mix<double>(const MixArgs &, const double *const *, double *const *, int, hipStream_t);
template void launch_mix<float>(const MixArgs &, const float *const *, float *const *, int, hipStream_t);
template void launch_env_init<double>(double *const *, int, int64_t, hipStream_t);
template void launch_env_init<float>(float *const *, int, int64_t, hipStream_t);
template void launch_env_final<double>(const double *const *, const double *const *, const int64_t *,
                                       const int *, const int64_t *, int, int, double *, int, hipStream_t);
template void launch_env_final<float>(const double *const *, const float *const *, const int64_t *,
                                      const int *, const int64_t *, int, int, double *, int, hipStream_t);
template void launch_repack<double>(const double *const *, double *const *, const int2 *, const int2 *,
                                    const int *, int, const int2 *, const int2 *, int, int, int, hipStream_t);
template void launch_repack<float>(const double *const *, float *const *, const int2 *, const int2 *,
                                   const int *, int, const int2 *, const int2 *, int, int, int, hipStream_t);

}  // namespace tnqe
