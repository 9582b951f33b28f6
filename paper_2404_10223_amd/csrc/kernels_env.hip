// Environment sweep on gfx950: block GEMMs (L x ket and bra^T x Y), the
// channel mix with the MPO (sparse rows and dense coupling GEMMs), and the
// compensated final element.
//
// Every pair keeps its own exact sector dimensions.  A block of the
// environment at bond b, for MPO channel class c (shift d = bra sector - ket
// sector) and ket sector s, is dense [dim_bra(s + d)][n_channels(c)]
// [dim_ket(s)] with the pair's dimensions; its slot in the pair's buffer is
// sized for the largest dimensions over all pairs, so one descriptor list
// (and one offset per block) serves every pair.  A launch runs over a work
// list of (descriptor, pair) entries holding only the tiles inside that
// pair's extents; a workgroup finds its entry by binary search.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"

namespace tnqe {

namespace {

template <typename T>
struct Seg {
  const T *A;
  const T *B;
  int K, lda, ldb, transA;   // A[m*lda + k] (transA 0) or A[k*lda + m]; B[k*ldb + n]
};

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 matrix-core step in FP64 or FP32 and the row of accumulator
// element r in lane j + 16 q: D[4 r + q][j] for v_mfma_f64_16x16x4f64,
// D[4 q + r][j] for v_mfma_f32_16x16x4f32 (both read A[i][k] from lane
// i + 16 k and B[k][j] from lane j + 16 k; layouts checked on gfx950).
template <typename V> struct Mfma;
template <> struct Mfma<double> {
  typedef v4d Acc;
  __device__ static Acc step(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int r, int q) { return 4 * r + q; }
};
template <> struct Mfma<float> {
  typedef v4f Acc;
  __device__ static Acc step(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int r, int q) { return 4 * q + r; }
};

// BF16 compute on FP32 operands (CM = 1: the operands rounded to BF16; CM = 2:
// each operand split as hi + lo, hi = bf16(x), lo = bf16(x - hi), and the
// product taken as hi hi + hi lo + lo hi), FP32 accumulation, one
// v_mfma_f32_16x16x16_bf16 per product and K chunk of 16: lane i + 16 q takes
// A[i][4 q .. 4 q + 3] and B[4 q .. 4 q + 3][i]; accumulator rows as for the
// FP32 instruction (D[4 q + r][j] in lane j + 16 q).
typedef short v4s __attribute__((ext_vector_type(4)));
__device__ inline unsigned short bf16_bits(float x) {   // round to nearest even
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_value(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Matrix-core tile (FP64 or FP32, V): the TM x TN tile (m0, n0) of sum over
// segments of A_q B_q, 256 threads = 4 waves, each wave a (TM / WM) x
// (TN / WN) sub-tile of 16 x 16 blocks accumulated by the 16 x 16 x 4
// instruction; K staged through LDS in chunks of 16.  la(q, m, k) /
// lb(q, k, n) load the operands of segment q (K of segment q: kq(q));
// sc(m, n, v) stores.  The loads of the next K chunk are issued before the
// current chunk's products.
template <typename V, int TM, int TN, int NSEG, int CM = 0, class KQ, class LA, class LB, class SC>
__device__ void tile_gemm_mfma(int M, int N, int m0, int n0, int nseg, KQ kq, LA la, LB lb, SC sc) {
  static_assert(CM == 0 || std::is_same<V, float>::value, "BF16 compute takes FP32 operands");
  constexpr int KC = 16;
  typedef typename Mfma<V>::Acc Acc;
  constexpr int WM = TM == TN ? 2 : (TM > TN ? 4 : 1), WN = 4 / WM;
  constexpr int SM = TM / WM, SN = TN / WN, BI = SM / 16, BJ = SN / 16;
  static_assert(BI >= 1 && BJ >= 1 && SM % 16 == 0 && SN % 16 == 0, "tile");
  __shared__ V sA[KC][TM + 1];
  __shared__ V sB[KC][TN + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave / WN) * SM, wn = (wave % WN) * SN;
  const int li = lane & 15, lk = lane >> 4;
  Acc acc[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) acc[i][j] = Acc{V(0), V(0), V(0), V(0)};
  // the next K chunk is loaded into registers while the current one is
  // multiplied (one chunk of global loads in flight per thread)
  constexpr int RA = KC * TM / 256, RB = KC * TN / 256;
  static_assert(RA * 256 == KC * TM && RB * 256 == KC * TN, "tile");
  V ra[RA], rb[RB];
  auto fetch = [&](int q, int K, int k0) {
#pragma unroll
    for (int u = 0; u < RA; ++u) {
      const int e = threadIdx.x + 256 * u, kk = e % KC, mm = e / KC;
      const int gm = m0 + mm, gk = k0 + kk;
      ra[u] = (gm < M && gk < K) ? la(q, gm, gk) : V(0);
    }
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int e = threadIdx.x + 256 * u, kk = e / TN, nn = e % TN;
      const int gn = n0 + nn, gk = k0 + kk;
      rb[u] = (gn < N && gk < K) ? lb(q, gk, gn) : V(0);
    }
  };
#pragma unroll
  for (int q = 0; q < NSEG; ++q) {
    if (q >= nseg) break;
    const int K = kq(q);
    if (K > 0) fetch(q, K, 0);
    for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
      for (int u = 0; u < RA; ++u) {
        const int e = threadIdx.x + 256 * u;
        sA[e % KC][e / KC] = ra[u];
      }
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int e = threadIdx.x + 256 * u;
        sB[e / TN][e % TN] = rb[u];
      }
      __syncthreads();
      if (k0 + KC < K) fetch(q, K, k0 + KC);
      if constexpr (CM == 0) {
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
          V a[BI], b[BJ];
#pragma unroll
          for (int i = 0; i < BI; ++i) a[i] = sA[ks + lk][wm + 16 * i + li];
#pragma unroll
          for (int j = 0; j < BJ; ++j) b[j] = sB[ks + lk][wn + 16 * j + li];
#pragma unroll
          for (int i = 0; i < BI; ++i)
#pragma unroll
            for (int j = 0; j < BJ; ++j) acc[i][j] = Mfma<V>::step(a[i], b[j], acc[i][j]);
        }
      } else {
        v4s ah[BI], bh[BJ], al[BI], bl[BJ];
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float x = sA[4 * lk + e][wm + 16 * i + li];
            const unsigned short h = bf16_bits(x);
            ah[i][e] = (short)h;
            al[i][e] = (short)bf16_bits(x - bf16_value(h));
          }
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float x = sB[4 * lk + e][wn + 16 * j + li];
            const unsigned short h = bf16_bits(x);
            bh[j][e] = (short)h;
            bl[j][e] = (short)bf16_bits(x - bf16_value(h));
          }
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
          for (int j = 0; j < BJ; ++j) {
            v4f c = acc[i][j];
            if constexpr (CM == 2) {
              c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[i], bh[j], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bl[j], c, 0, 0, 0);
            }
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bh[j], c, 0, 0, 0);
          }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + 16 * i + Mfma<V>::row(r, lk), gn = n0 + wn + 16 * j + li;
        if (gm < M && gn < N) sc(gm, gn, acc[i][j][r]);
      }
}

// C tile (m0, n0) of sum_seg op(A) B on the matrix cores (tile_gemm_mfma, in
// the precision of T).  C = alpha * sum (+ C if beta).
template <typename T, int TM, int TN, int RM, int RN, int NSEG, int CM>
__device__ void tile_gemm(int M, int N, int m0, int n0, const Seg<T> (&sg)[NSEG], int nseg, T *C, int ldc,
                          T alpha, int beta) {
  tile_gemm_mfma<T, TM, TN, NSEG, CM>(
      M, N, m0, n0, nseg, [&](int q) { return sg[q].K; },
      [&](int q, int m, int k) {
        const Seg<T> &s = sg[q];
        return s.transA ? s.A[(int64_t)k * s.lda + m] : s.A[(int64_t)m * s.lda + k];
      },
      [&](int q, int k, int n) { return sg[q].B[(int64_t)k * sg[q].ldb + n]; },
      [&](int m, int n, T v) {
        T *c = C + (int64_t)m * ldc + n;
        *c = beta ? *c + alpha * v : alpha * v;
      });
}

// the work entry owning workgroup wg: last entry with first <= wg
__device__ inline EnvWork find_work(const EnvWork *work, int nwork, int wg) {
  int lo = 0, hi = nwork - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (work[mid].first <= wg) lo = mid; else hi = mid - 1;
  }
  return work[lo];
}

// X[(c, s, k)] = L[(c, s)] A_ket[s, k, s + q(k)]
template <typename T, int TM, int TN, int RM, int RN, int CM>
__global__ void __launch_bounds__(256) k_env_g1(const EnvG1 *descs, const EnvWork *work, int nwork, EnvGeom g,
                                                const T *const *L, const T *const *ket, T *const *X) {
  const EnvWork w = find_work(work, nwork, blockIdx.x);
  const int pair = w.pair;
  const EnvG1 d = descs[w.desc];
  const int bi = g.bra[pair], ki = g.ket[pair];
  const int dbra = g.sec(bi, d.x, d.sbra).y;
  const int2 sk = g.sec(ki, d.x, d.s), sn = g.sec(ki, d.x + 1, d.sk);
  const int M = dbra * d.nw, N = sn.y;
  const int t = blockIdx.x - w.first, tilesN = (N + TN - 1) / TN;
  const int m0 = (t / tilesN) * TM, n0 = (t % tilesN) * TN;
  if (m0 >= M || n0 >= N) return;
  const int Dr = g.dim(ki, d.x + 1);
  Seg<T> sg[1];
  sg[0].A = L[pair] + d.offL;
  sg[0].lda = sk.y;
  sg[0].transA = 0;
  sg[0].B = ket[pair] + ((int64_t)sk.x * 4 + d.k) * Dr + sn.x;
  sg[0].ldb = 4 * Dr;
  sg[0].K = sk.y;
  tile_gemm<T, TM, TN, RM, RN, 1, CM>(M, N, m0, n0, sg, 1, X[pair] + d.offX, N, T(1), 0);
}

// L'[(c, s)] = sum_k' A_bra[s_a(k'), k', s + d]^T Y[(c, s, k')]
template <typename T, int TM, int TN, int RM, int RN, int CM>
__global__ void __launch_bounds__(256) k_env_g2(const EnvG2 *descs, const EnvWork *work, int nwork, EnvGeom g,
                                                const T *const *bra, const T *const *Y, T *const *Ln) {
  const EnvWork w = find_work(work, nwork, blockIdx.x);
  const int pair = w.pair;
  const EnvG2 d = descs[w.desc];
  const int bi = g.bra[pair], ki = g.ket[pair];
  const int2 sbn = g.sec(bi, d.x + 1, d.sbn);
  const int M = sbn.y, N = d.nw * g.sec(ki, d.x + 1, d.s).y;
  const int t = blockIdx.x - w.first, tilesN = (N + TN - 1) / TN;
  const int m0 = (t / tilesN) * TM, n0 = (t % tilesN) * TN;
  if (m0 >= M || n0 >= N) return;
  const int Dr = g.dim(bi, d.x + 1);
  Seg<T> sg[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int2 sa = g.sec(bi, d.x, q < d.nseg ? d.sa[q] : -1);
    sg[q].A = bra[pair] + ((int64_t)sa.x * 4 + d.kp[q]) * Dr + sbn.x;
    sg[q].lda = 4 * Dr;
    sg[q].transA = 1;
    sg[q].B = Y[pair] + d.offY[q];
    sg[q].ldb = N;
    sg[q].K = q < d.nseg ? sa.y : 0;
  }
  tile_gemm<T, TM, TN, RM, RN, 4, CM>(M, N, m0, n0, sg, d.nseg, Ln[pair] + d.offL, N, T(1), 0);
}

// C tile (m0, n0) of A B with element loaders (A: m x k, B: k x n) and an
// accumulating store; same tiling as tile_gemm.
template <typename T, int TM, int TN, int RM, int RN, int CM, class LA, class LB, class SC>
__device__ void tile_gemm_f(int M, int N, int K, int m0, int n0, LA la, LB lb, SC sc) {
  tile_gemm_mfma<T, TM, TN, 1, CM>(
      M, N, m0, n0, 1, [&](int) { return K; }, [&](int, int m, int k) { return la(m, k); },
      [&](int, int k, int n) { return lb(k, n); }, sc);
}

// dense channel coupling: Y[a][r0 + i][b] += f sum_j W[i][j] X[a][c0 + j][b],
// one GEMM over all bra rows a of the block: M = nr, K = nc, N = (a, b)
template <typename T, int TM, int TN, int RM, int RN, int CM>
__global__ void __launch_bounds__(256) k_env_gd(const EnvGD *descs, const EnvWork *work, int nwork, EnvGeom g,
                                                const T *const *vals, const T *const *X, T *const *Y) {
  const EnvWork w = find_work(work, nwork, blockIdx.x);
  const int pair = w.pair;
  const EnvGD d = descs[w.desc];
  const int bi = g.bra[pair], ki = g.ket[pair];
  const int da = g.sec(bi, d.x, d.sa).y, db = g.sec(ki, d.x + 1, d.s).y;
  const int N = da * db;
  const int t = blockIdx.x - w.first, tilesN = (N + TN - 1) / TN;
  const int m0 = (t / tilesN) * TM, n0 = (t % tilesN) * TN;
  if (m0 >= d.nr || n0 >= N) return;
  const T *W = vals[pair] + d.valoff;
  const T *Xb = X[pair] + d.offX + (int64_t)d.c0 * db;
  T *Yb = Y[pair] + d.offY + (int64_t)d.r0 * db;
  const int nc = d.nc, xs = d.nw_in * db, ys = d.nw_out * db;
  const T f = (T)d.f;
  tile_gemm_f<T, TM, TN, RM, RN, CM>(
      d.nr, N, nc, m0, n0, [&](int m, int k) { return W[(int64_t)m * nc + k]; },
      [&](int k, int n) {
        const int a = n / db, b = n - a * db;
        return Xb[(int64_t)a * xs + (int64_t)k * db + b];
      },
      [&](int m, int n, T v) {
        const int a = n / db, b = n - a * db;
        T *y = Yb + (int64_t)a * ys + (int64_t)m * db + b;
        *y += f * v;
      });
}

// ------------------------------------------------------------------ channel mix
// Y[a][w'][b] = sum over the task's sources and the nonzeros z of row w' of
// each source's MPO group of factor * v_z * X[a][col_z][b].  A thread takes
// RA = kMixRows consecutive bra rows a of one output channel w' and CJ =
// kMixCols ket columns b = t + j qpr (j < CJ, qpr = ceil(db / CJ)); the qpr
// threads of a (rows, w') group are consecutive, so each load and store
// instruction covers contiguous columns across the group's lanes, and each
// coupling a thread loads serves all its rows and columns.  The loads of
// kMixUnroll couplings are issued together.
template <typename T>
__global__ void __launch_bounds__(256) k_mix(MixArgs a, EnvGeom g, const T *const *X, T *const *Y) {
  constexpr int RA = kMixRows, CJ = kMixCols, U = kMixUnroll;
  const EnvWork wk = find_work(a.work, a.nwork, blockIdx.x);
  const int pair = wk.pair;
  const MixTask tk = a.tasks[wk.desc];
  const int da = g.sec(g.bra[pair], tk.x, tk.sa).y, db = g.sec(g.ket[pair], tk.x + 1, tk.s).y;
  const int qpr = (db + CJ - 1) / CJ, nag = (da + RA - 1) / RA;
  const int item = (blockIdx.x - wk.first) * 256 + threadIdx.x;
  if (item >= nag * tk.nw_out * qpr) return;
  const int row = item / qpr, b0 = item - row * qpr;
  const int ag = row / tk.nw_out, w = row - ag * tk.nw_out;
  const int ap0 = ag * RA, na = min(RA, da - ap0);
  const double *vals = a.vals + a.basis[pair] * a.basis_stride;
  const T *Xp = X[pair];
  // columns b0 + j qpr, j < nb, lie inside the block
  const int nb = (db - b0 + qpr - 1) / qpr;
  double acc[RA][CJ] = {};
  for (int si = tk.src0; si < tk.src0 + tk.nsrc; ++si) {
    const MixSrc sr = a.srcs[si];
    const int z0 = a.rowptr[sr.rp + w], z1 = a.rowptr[sr.rp + w + 1];
    const int *col = a.col + sr.cp;
    const double *v = vals + sr.vbase;
    const int64_t rs = (int64_t)sr.nw_in * db;   // X row stride between bra rows
    const T *xb = Xp + sr.offX + (int64_t)ap0 * rs + b0;
    // U couplings at a time: their loads (all rows) are issued together;
    // the terms are added in coupling order
    int z = z0;
    for (; z + U <= z1; z += U) {
      double cf[U], xv[U][RA][CJ];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        cf[u] = sr.factor * v[z + u];
        const T *xr = xb + (int64_t)col[z + u] * db;
#pragma unroll
        for (int r = 0; r < RA; ++r)
#pragma unroll
          for (int j = 0; j < CJ; ++j) xv[u][r][j] = (r < na && j < nb) ? (double)xr[r * rs + j * qpr] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < RA; ++r)
#pragma unroll
          for (int j = 0; j < CJ; ++j) acc[r][j] += cf[u] * xv[u][r][j];
    }
    for (; z < z1; ++z) {
      const double cf = sr.factor * v[z];
      const T *xr = xb + (int64_t)col[z] * db;
#pragma unroll
      for (int r = 0; r < RA; ++r)
#pragma unroll
        for (int j = 0; j < CJ; ++j)
          if (r < na && j < nb) acc[r][j] += cf * (double)xr[r * rs + j * qpr];
    }
  }
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    if (r >= na) break;
    T *yr = Y[pair] + tk.offY + ((int64_t)(ap0 + r) * tk.nw_out + w) * db + b0;
#pragma unroll
    for (int j = 0; j < CJ; ++j)
      if (j < nb) yr[j * qpr] = (T)acc[r][j];
  }
}

template <typename T>
struct Pair2;
template <>
struct Pair2<double> {
  typedef double2 type;
};
template <>
struct Pair2<float> {
  typedef float2 type;
};

// The channel mix of the task-pairs with an even number db of ket columns: a
// thread takes kMix2Rows consecutive bra rows of one output channel and the
// column pair (2t, 2t + 1), loaded and stored as one vector (the offsets of
// every X and Y block, and with db even every row, are even).  Terms in the
// order of k_mix.
template <typename T>
__global__ void __launch_bounds__(256) k_mix2(MixArgs a, EnvGeom g, const T *const *X, T *const *Y) {
  constexpr int RA = kMix2Rows, U = kMixUnroll;
  typedef typename Pair2<T>::type T2;
  const EnvWork wk = find_work(a.work, a.nwork, blockIdx.x);
  const int pair = wk.pair;
  const MixTask tk = a.tasks[wk.desc];
  const int da = g.sec(g.bra[pair], tk.x, tk.sa).y, db = g.sec(g.ket[pair], tk.x + 1, tk.s).y;
  const int qpr = db >> 1, nag = (da + RA - 1) / RA;
  const int item = (blockIdx.x - wk.first) * 256 + threadIdx.x;
  if (item >= nag * tk.nw_out * qpr) return;
  const int row = item / qpr, b = 2 * (item - row * qpr);
  const int ag = row / tk.nw_out, w = row - ag * tk.nw_out;
  const int ap0 = ag * RA, na = min(RA, da - ap0);
  const double *vals = a.vals + a.basis[pair] * a.basis_stride;
  const T *Xp = X[pair];
  double acc[RA][2] = {};
  for (int si = tk.src0; si < tk.src0 + tk.nsrc; ++si) {
    const MixSrc sr = a.srcs[si];
    const int z0 = a.rowptr[sr.rp + w], z1 = a.rowptr[sr.rp + w + 1];
    const int *col = a.col + sr.cp;
    const double *v = vals + sr.vbase;
    const int64_t rs = (int64_t)sr.nw_in * db;   // X row stride between bra rows
    const T *xb = Xp + sr.offX + (int64_t)ap0 * rs + b;
    int z = z0;
    for (; z + U <= z1; z += U) {
      double cf[U];
      T2 xv[U][RA];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        cf[u] = sr.factor * v[z + u];
        const T *xr = xb + (int64_t)col[z + u] * db;
#pragma unroll
        for (int r = 0; r < RA; ++r)
          xv[u][r] = r < na ? *reinterpret_cast<const T2 *>(xr + r * rs) : T2{T(0), T(0)};
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < RA; ++r) {
          acc[r][0] += cf[u] * (double)xv[u][r].x;
          acc[r][1] += cf[u] * (double)xv[u][r].y;
        }
    }
    for (; z < z1; ++z) {
      const double cf = sr.factor * v[z];
      const T *xr = xb + (int64_t)col[z] * db;
#pragma unroll
      for (int r = 0; r < RA; ++r)
        if (r < na) {
          const T2 xv = *reinterpret_cast<const T2 *>(xr + r * rs);
          acc[r][0] += cf * (double)xv.x;
          acc[r][1] += cf * (double)xv.y;
        }
    }
  }
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    if (r >= na) break;
    T *yr = Y[pair] + tk.offY + ((int64_t)(ap0 + r) * tk.nw_out + w) * db + b;
    *reinterpret_cast<T2 *>(yr) = T2{(T)acc[r][0], (T)acc[r][1]};
  }
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

// last site: out[pair * nw + w] = sum_{k', a'} bra[a', k', 0] Y_k'[a'][w][0],
// accumulated with TwoSum and a compensated tree
template <typename T>
__global__ void __launch_bounds__(256) k_env_final(EnvGeom g, int x, const double *const *bra, const T *const *Y,
                                                   const EnvFinal *fin, int nk, int nw, double *out) {
  const int pair = blockIdx.x;
  const int bi = g.bra[pair];
  __shared__ double ss[256], se[256];
  for (int w = 0; w < nw; ++w) {
    double s = 0.0, c = 0.0;
    for (int k = 0; k < nk; ++k) {
      const int2 sa = g.sec(bi, x, fin[k].sa);
      const T *y = Y[pair] + fin[k].offY;
      // bra index i of the sector, local state k': bra[(off + i) * 4 + k'] (right bond 1)
      const double *bp = bra[pair] + (int64_t)sa.x * 4 + fin[k].kp;
      for (int i = threadIdx.x; i < sa.y; i += 256) {
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

// dst[i][e] = (float) src[i][e] for e < count[i]
__global__ void k_cast(const double *const *src, float *const *dst, const int64_t *count) {
  const int i = blockIdx.y;
  const int64_t n = count[i];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[i][e] = (float)src[i][e];
}

// y[b][j] = x[b][j] + a z[j] for every basis b (nnz entries each)
__global__ void k_shift_vals(const double *x, const double *z, double a, int64_t nnz, double *y) {
  const int64_t b = blockIdx.y;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * blockDim.x)
    y[b * nnz + j] = x[b * nnz + j] + a * z[j];
}

// ------------------------------------------------------------ one-hot pencil
// Dense contractions of the expanded one-hot pencil (App. A1): the index maps
// of each kind are listed with OhGemm.
__device__ inline double oh_la(const OhGemm &g, int m, int k) {
  switch (g.kind) {
    case kOhPlainAT:
    case kOhBraL:
      return g.A[(int64_t)k * g.M + m];
    case kOhWX:
    case kOhA3: {
      const int wo = m >> 2, ko = m & 3, wi = k >> 2, ki = k & 3;
      return g.A[(((int64_t)wi * g.d0 + wo) * 4 + ko) * 4 + ki];
    }
    case kOhRX2: {
      const int w = m >> 2, kp = m & 3, w2 = k >> 2, kk = k & 3;
      return g.A[(((int64_t)w * g.d0 + w2) * 4 + kp) * 4 + kk];
    }
    case kOhA4: {
      const int l = m >> 4, kp = (m >> 2) & 3, kq = m & 3, w2 = k / g.d1, b = k - w2 * g.d1;
      return g.A[((int64_t)w2 * 4 + kq) * (4 * (int64_t)g.d0 * g.d1) + ((int64_t)kp * g.d0 + l) * g.d1 + b];
    }
    case kOhD1:
      return g.A[((int64_t)(m >> 4) * g.d0 + k) * 16 + (m & 15)];
    case kOhD3: {
      const int ll2 = m >> 8, kpkp2 = (m >> 4) & 15, kqkq2 = m & 15;
      return g.A[(int64_t)ll2 * (256 * (int64_t)g.d1) + ((int64_t)kpkp2 * g.d1 + k) * 16 + kqkq2];
    }
    default:   // Plain, PlainBT, BraR
      return g.A[(int64_t)m * g.K + k];
  }
}

__device__ inline double oh_lb(const OhGemm &g, int k, int n) {
  switch (g.kind) {
    case kOhPlainBT:
      return g.B[(int64_t)n * g.K + k];
    case kOhWX: {
      const int wi = k >> 2, ki = k & 3, a = n / g.d2, x = n - a * g.d2;
      return g.B[(((int64_t)wi * g.d1 + a) * 4 + ki) * g.d2 + x];
    }
    case kOhBraL: {
      const int a = k >> 2, kp = k & 3, w = n / g.d1, b = n - w * g.d1;
      return g.B[(((int64_t)w * 4 + kp) * g.d0 + a) * g.d1 + b];
    }
    case kOhRX2:
      return g.B[((int64_t)(k >> 2) * g.N + n) * 4 + (k & 3)];
    case kOhBraR: {
      const int w = n / g.d0, a = n - w * g.d0;
      return g.B[((int64_t)w * g.K + k) * g.d0 + a];
    }
    case kOhA3: {
      const int w1 = k >> 2, kq2 = k & 3, kp = n / (g.d1 * g.d2), rest = n - kp * g.d1 * g.d2;
      const int l = rest / g.d2, b = rest - l * g.d2;
      return g.B[((int64_t)w1 * 4 + kp) * (4 * (int64_t)g.d1 * g.d2) + ((int64_t)l * 4 + kq2) * g.d2 + b];
    }
    case kOhA4: {
      const int w2 = k / g.d1, b = k - w2 * g.d1;
      return g.B[((int64_t)w2 * g.d2 + n) * g.d1 + b];
    }
    default:   // Plain, PlainAT, D1, D3
      return g.B[(int64_t)k * g.N + n];
  }
}

__device__ inline void oh_st(const OhGemm &g, int m, int n, double v) {
  switch (g.kind) {
    case kOhBraL: {
      const int w = n / g.d1, b = n - w * g.d1;
      g.C[((int64_t)w * g.M + m) * g.d1 + b] = v;
      return;
    }
    case kOhBraR: {
      const int w = n / g.d0, a = n - w * g.d0;
      g.C[((int64_t)w * g.M + m) * g.d0 + a] = v;
      return;
    }
    case kOhD3: {
      const int ll2 = m >> 8, kp = (m >> 6) & 3, kp2 = (m >> 4) & 3, kq = (m >> 2) & 3, kq2 = m & 3;
      const int l = ll2 / g.d0, l2 = ll2 - l * g.d0, r = n / g.d2, r2 = n - r * g.d2;
      const int row = g.map[(((int64_t)l * 4 + kp) * 4 + kq) * g.d2 + r];
      const int col = g.map[(((int64_t)l2 * 4 + kp2) * 4 + kq2) * g.d2 + r2];
      if (row >= 0 && col >= 0) g.C[(int64_t)row * g.n_oh + col] = v;
      return;
    }
    default:
      g.C[(int64_t)m * g.N + n] = v;
  }
}

__global__ void __launch_bounds__(256) k_oh_gemm(OhGemm g) {
  const int tilesN = (g.N + 63) / 64;
  const int m0 = (blockIdx.x / tilesN) * 64, n0 = (blockIdx.x % tilesN) * 64;
  tile_gemm_mfma<double, 64, 64, 1>(
      g.M, g.N, m0, n0, 1, [&](int) { return g.K; }, [&](int, int m, int k) { return oh_la(g, m, k); },
      [&](int, int k, int n) { return oh_lb(g, k, n); }, [&](int m, int n, double v) { oh_st(g, m, n, v); });
}

__global__ void k_oh_gather(const double *V, const double *S, double f, const int *idx, int n, double *out, int ld,
                            int col) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  out[(int64_t)m * ld + col] = V[idx[m]] + (S ? f * S[idx[m]] : 0.0);
}

__global__ void k_oh_sd(const int4 *oh, int n, const double *LS, int Db, const double *RS, int Db2, double e_core,
                        double *Sd, double *Hd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int4 a = oh[e / n], b = oh[e % n];
  const double v = (a.y == b.y && a.z == b.z) ? LS[(int64_t)a.x * Db + b.x] * RS[(int64_t)a.w * Db2 + b.w] : 0.0;
  Sd[e] = v;
  Hd[e] += e_core * v;
}

}  // namespace

#define TNQE_TILE_SWITCH(KERNEL, T, CM, tileM, tileN, grid, ...)                               \
  do {                                                                                         \
    if (tileM == 256 && tileN == 16)                                                           \
      hipLaunchKernelGGL((KERNEL<T, 256, 16, 16, 1, CM>), grid, dim3(256), 0, __VA_ARGS__);    \
    else if (tileM == 16 && tileN == 256)                                                      \
      hipLaunchKernelGGL((KERNEL<T, 16, 256, 1, 16, CM>), grid, dim3(256), 0, __VA_ARGS__);    \
    else if (tileM == 128 && tileN == 32)                                                      \
      hipLaunchKernelGGL((KERNEL<T, 128, 32, 8, 2, CM>), grid, dim3(256), 0, __VA_ARGS__);     \
    else if (tileM == 32 && tileN == 128)                                                      \
      hipLaunchKernelGGL((KERNEL<T, 32, 128, 2, 8, CM>), grid, dim3(256), 0, __VA_ARGS__);     \
    else                                                                                       \
      hipLaunchKernelGGL((KERNEL<T, 64, 64, 4, 4, CM>), grid, dim3(256), 0, __VA_ARGS__);      \
  } while (0)

// compute mode cm (FP32 storage only): 0 native, 1 BF16, 2 split BF16
#define TNQE_CM_SWITCH(KERNEL, T, cm, tileM, tileN, grid, ...)                                 \
  do {                                                                                         \
    if constexpr (std::is_same<T, float>::value) {                                             \
      if (cm == 1) { TNQE_TILE_SWITCH(KERNEL, T, 1, tileM, tileN, grid, __VA_ARGS__); break; } \
      if (cm == 2) { TNQE_TILE_SWITCH(KERNEL, T, 2, tileM, tileN, grid, __VA_ARGS__); break; } \
    }                                                                                          \
    TNQE_TILE_SWITCH(KERNEL, T, 0, tileM, tileN, grid, __VA_ARGS__);                           \
  } while (0)

template <typename T>
void launch_env_g1(const EnvG1 *d, const EnvWork *work, int nwork, int nwg, int tileM, int tileN,
                   const EnvGeom &g, const T *const *L, const T *const *ket, T *const *X, hipStream_t st, int cm) {
  if (nwork == 0 || nwg == 0) return;
  TNQE_CM_SWITCH(k_env_g1, T, cm, tileM, tileN, dim3(nwg), st, d, work, nwork, g, L, ket, X);
}

template <typename T>
void launch_env_g2(const EnvG2 *d, const EnvWork *work, int nwork, int nwg, int tileM, int tileN,
                   const EnvGeom &g, const T *const *bra, const T *const *Y, T *const *Ln, hipStream_t st, int cm) {
  if (nwork == 0 || nwg == 0) return;
  TNQE_CM_SWITCH(k_env_g2, T, cm, tileM, tileN, dim3(nwg), st, d, work, nwork, g, bra, Y, Ln);
}

template <typename T>
void launch_env_gd(const EnvGD *d, const EnvWork *work, int nwork, int nwg, int tileM, int tileN,
                   const EnvGeom &g, const T *const *vals, const T *const *X, T *const *Y, hipStream_t st, int cm) {
  if (nwork == 0 || nwg == 0) return;
  TNQE_CM_SWITCH(k_env_gd, T, cm, tileM, tileN, dim3(nwg), st, d, work, nwork, g, vals, X, Y);
}

template <typename T>
void launch_mix(const MixArgs &a, const EnvGeom &g, const T *const *X, T *const *Y, hipStream_t st) {
  if (a.nwork == 0 || a.nchunk == 0) return;
  hipLaunchKernelGGL(k_mix<T>, dim3(a.nchunk), dim3(256), 0, st, a, g, X, Y);
}

template <typename T>
void launch_mix2(const MixArgs &a, const EnvGeom &g, const T *const *X, T *const *Y, hipStream_t st) {
  if (a.nwork == 0 || a.nchunk == 0) return;
  hipLaunchKernelGGL(k_mix2<T>, dim3(a.nchunk), dim3(256), 0, st, a, g, X, Y);
}

template <typename T>
void launch_env_init(T *const *L, int npair, int64_t size, hipStream_t st) {
  if (npair == 0) return;
  hipLaunchKernelGGL(k_env_init<T>, dim3(1, npair), dim3(64), 0, st, L, size);
}

template <typename T>
void launch_env_final(const EnvGeom &g, int x, const double *const *bra, const T *const *Y, const EnvFinal *fin,
                      int nk, int nw, double *out, int npair, hipStream_t st) {
  if (npair == 0) return;
  hipLaunchKernelGGL(k_env_final<T>, dim3(npair), dim3(256), 0, st, g, x, bra, Y, fin, nk, nw, out);
}

void launch_oh_gemm(const OhGemm &g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  const int64_t tiles = (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64);
  if (tiles >= (int64_t)1 << 31) throw Error(TNQE_ESHAPE, "one-hot contraction too large");
  hipLaunchKernelGGL(k_oh_gemm, dim3((unsigned)tiles), dim3(256), 0, st, g);
}

void launch_oh_gather(const double *V, const double *S, double f, const int *idx, int n, double *out, int ld, int col,
                      hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_oh_gather, dim3((n + 255) / 256), dim3(256), 0, st, V, S, f, idx, n, out, ld, col);
}

void launch_oh_sd(const int4 *oh, int n, const double *LS, int Db, const double *RS, int Db2, double e_core,
                  double *Sd, double *Hd, hipStream_t st) {
  const int64_t tot = (int64_t)n * n;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_oh_sd, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, oh, n, LS, Db, RS, Db2, e_core,
                     Sd, Hd);
}

void launch_shift_vals(const double *x, const double *z, double a, int64_t nnz, int nbasis, double *y,
                       hipStream_t st) {
  if (nnz == 0 || nbasis == 0) return;
  hipLaunchKernelGGL(k_shift_vals, dim3(64, nbasis), dim3(256), 0, st, x, z, a, nnz, y);
}

void launch_cast(const double *const *src, float *const *dst, const int64_t *count, int n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_cast, dim3(64, n), dim3(256), 0, st, src, dst, count);
}

#define TNQE_ENV_INST(T)                                                                                     \
  template void launch_env_g1<T>(const EnvG1 *, const EnvWork *, int, int, int, int, const EnvGeom &,       \
                                 const T *const *, const T *const *, T *const *, hipStream_t, int);         \
  template void launch_env_g2<T>(const EnvG2 *, const EnvWork *, int, int, int, int, const EnvGeom &,       \
                                 const T *const *, const T *const *, T *const *, hipStream_t, int);         \
  template void launch_env_gd<T>(const EnvGD *, const EnvWork *, int, int, int, int, const EnvGeom &,       \
                                 const T *const *, const T *const *, T *const *, hipStream_t, int);         \
  template void launch_mix<T>(const MixArgs &, const EnvGeom &, const T *const *, T *const *, hipStream_t); \
  template void launch_mix2<T>(const MixArgs &, const EnvGeom &, const T *const *, T *const *, hipStream_t); \
  template void launch_env_init<T>(T *const *, int, int64_t, hipStream_t);                                  \
  template void launch_env_final<T>(const EnvGeom &, int, const double *const *, const T *const *,          \
                                    const EnvFinal *, int, int, double *, int, hipStream_t);
TNQE_ENV_INST(double)
TNQE_ENV_INST(float)

}  // namespace tnqe
