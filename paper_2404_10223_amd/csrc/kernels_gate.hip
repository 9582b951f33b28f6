// Gate phase on gfx950: two-site gate contraction, split of the truncated
// factors, and exact centre moves (the SVDs are in kernels_svd.hip).
//
// Every kernel works on a list of quantum-number blocks.  Blocks of all kets
// in flight are launched together, so one launch covers every pair of the
// subspace at the same gate position; the blocks are cut into work units
// (output tiles or element chunks, one workgroup each) so that the few large
// blocks of a launch do not leave most compute units idle.  Site tensors
// are stored dense, but every kernel (and the environment sweep) addresses
// them by quantum-number block, so entries outside the blocks are never read
// and are not cleared when a bond changes.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace tnqe {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// The block descriptor of a workgroup, staged in LDS: the segment tables are
// indexed with run-time indices, which would put a register copy of the
// descriptor in per-lane scratch memory.
__device__ const Blk &stage_block(const Blk *blks, int i) {
  __shared__ Blk s_blk;
  if (threadIdx.x == 0) s_blk = blks[i];
  __syncthreads();
  return s_blk;
}

__device__ inline int seg_of(const int *s, int x) {
  int k = 0;
  while (k < 3 && x >= s[k + 1]) ++k;
  return k;
}

// One 64 x 64 tile (rows m0.., columns n0..) of an M x N product C = A B
// (4 x 4 per thread, K through LDS in steps of 16, the next step's loads
// issued before the current step's products); la(m, k) and lb(k, n) load
// operands, sc(m, n, v) stores.  A tiles are filled with k fastest; B tiles
// with k fastest when BK (B contiguous along k), else with n fastest.
constexpr int kKC = 16;
typedef double GemmTile[kKC][kGateTile + 1];
template <bool BK, class LA, class LB, class SC>
__device__ void gemm_tile(GemmTile &sA, GemmTile &sB, int M, int N, int K, int m0, int n0, LA la, LB lb,
                          SC sc) {
  constexpr int TT = kGateTile, KC = kKC, R = KC * TT / kThreads;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  // operands of the next K chunk are loaded into registers while the
  // current chunk is multiplied
  double ra[R], rb[R];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int e = threadIdx.x + kThreads * u;
      const int kk = e % KC, mm = e / KC;
      const int gm = m0 + mm, gk = k0 + kk;
      ra[u] = (gm < M && gk < K) ? la(gm, gk) : 0.0;
      if (BK) {
        const int gn = n0 + mm;
        rb[u] = (gn < N && gk < K) ? lb(gk, gn) : 0.0;
      } else {
        const int nn = e % TT, kb = e / TT;
        const int gn = n0 + nn, gkb = k0 + kb;
        rb[u] = (gn < N && gkb < K) ? lb(gkb, gn) : 0.0;
      }
    }
  };
  if (K > 0) fetch(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int e = threadIdx.x + kThreads * u;
      sA[e % KC][e / KC] = ra[u];
      if (BK) sB[e % KC][e / KC] = rb[u];
      else sB[e / TT][e % TT] = rb[u];
    }
    __syncthreads();
    if (k0 + KC < K) fetch(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = sA[kk][ty + 16 * u];
        bv[u] = sB[kk][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int gm = m0 + ty + 16 * u;
    if (gm >= M) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gn = n0 + tx + 16 * v;
      if (gn < N) sc(gm, gn, acc[u][v]);
    }
  }
}

// tile t of an M x N product (row-major tile order)
template <bool BK, class LA, class LB, class SC>
__device__ void gemm_tile_at(GemmTile &sA, GemmTile &sB, int M, int N, int K, int t, LA la, LB lb, SC sc) {
  const int tilesN = (N + kGateTile - 1) / kGateTile;
  gemm_tile<BK>(sA, sB, M, N, K, (t / tilesN) * kGateTile, (t % tilesN) * kGateTile, la, lb, sc);
}

// All tiles of a product in one workgroup (used where a launch has few,
// small blocks: the QR moves of the initial canonical form).
template <bool BK, class LA, class LB, class SC>
__device__ void block_gemm(int M, int N, int K, LA la, LB lb, SC sc) {
  __shared__ GemmTile sA, sB;
  const int nt = gate_tiles(M, N);
  for (int t = 0; t < nt; ++t) gemm_tile_at<BK>(sA, sB, M, N, K, t, la, lb, sc);
}

// Two-site product per old middle sector ms = (sa, sb) of bond a+1:
// Theta[(k1, l)][(k2, r)] = sum_m A_a[l, k1, m] A_{a+1}[m, k2, r], with l in
// the left sector ms - q(k1) and r in the right sector ms + q(k2).  One
// 64 x 64 output tile per workgroup.
__global__ void __launch_bounds__(kThreads) k_theta(KetTables kt, int a, const Blk *th, Units un,
                                                    double *scratch) {
  const int bi = find_unit(un.first, un.n, blockIdx.x);
  const int t = blockIdx.x - un.first[bi];
  const Blk &b = stage_block(th, bi);
  const int pair = b.pair;
  const double *A = kt.site[pair * kt.N + a];
  const double *B = kt.site[pair * kt.N + a + 1];
  const int Dm = kt.dim(a + 1, pair), Dr = kt.dim(a + 2, pair);
  const int2 mid = kt.sec(a + 1, pair, b.sa, b.sb);
  __shared__ int s_lo[4], s_ro[4];
  __shared__ GemmTile sA, sB;
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    s_lo[k] = kt.sec(a, pair, b.sa - qk_a(k), b.sb - qk_b(k)).x;
    s_ro[k] = kt.sec(a + 2, pair, b.sa + qk_a(k), b.sb + qk_b(k)).x;
  }
  __syncthreads();
  double *Th = scratch + b.offT;
  const int C = b.C;
  // A rows (k1, l) are contiguous along the middle index; B columns (k2, r)
  // along the right index
  gemm_tile_at<false>(
      sA, sB, b.R, C, mid.y, t,
      [&](int row, int m) {
        const int k1 = seg_of(b.rs, row);
        return A[((int64_t)(s_lo[k1] + row - b.rs[k1]) * 4 + k1) * Dm + mid.x + m];
      },
      [&](int m, int col) {
        const int k2 = seg_of(b.cs, col);
        return B[((int64_t)(mid.x + m) * 4 + k2) * Dr + s_ro[k2] + col - b.cs[k2]];
      },
      [&](int row, int col, double v) { Th[(int64_t)row * C + col] = v; });
}

// The 16 x 16 gate of every pair from (cos, sin) of its angle (one
// workgroup of 256 threads per pair).
__global__ void __launch_bounds__(256) k_gates(const double *cs, double *gates) {
  const int pair = blockIdx.x;
  gates[(int64_t)pair * 256 + threadIdx.x] = gate4_entry(cs[2 * pair], cs[2 * pair + 1], threadIdx.x);
}

// T'[(k1', l)][(k2', r)] = sum_{k1,k2} G[(k1',k2'),(k1,k2)] Theta_ms[(k1, l)][(k2, r)]
// with ms = s - q(k1') + q(k1) (the gate conserves both particle numbers, so
// the row and column sectors of the two sides agree).  thidx[pair][slot] is
// the Theta block of a middle sector (-1: none, the product is empty).
__global__ void __launch_bounds__(kThreads) k_gate_gather(KetTables kt, const Blk *blks, Units un,
                                                          const Blk *th, const int *thidx,
                                                          const double *gates, double *scratch) {
  const int bi = find_unit(un.first, un.n, blockIdx.x);
  const Blk &b = stage_block(blks, bi);
  const int64_t e0 = (int64_t)(blockIdx.x - un.first[bi]) * kGateChunk;
  const int pair = b.pair;
  __shared__ double sG[256];
  __shared__ int64_t s_off[16];
  __shared__ int s_C[16], s_rs[16][5], s_cs[16][5];
  for (int i = threadIdx.x; i < 256; i += kThreads) sG[i] = gates[(int64_t)pair * 256 + i];
  if (threadIdx.x < 16) {
    const int k1p = threadIdx.x >> 2, k1 = threadIdx.x & 3;
    const int slot = kt.slot(b.sa - qk_a(k1p) + qk_a(k1), b.sb - qk_b(k1p) + qk_b(k1));
    const int ti = slot < 0 ? -1 : thidx[pair * kt.nslot + slot];
    s_off[threadIdx.x] = -1;
    if (ti >= 0) {
      const Blk &t = th[ti];
      s_off[threadIdx.x] = t.offT;
      s_C[threadIdx.x] = t.C;
      for (int k = 0; k < 5; ++k) {
        s_rs[threadIdx.x][k] = t.rs[k];
        s_cs[threadIdx.x][k] = t.cs[k];
      }
    }
  }
  __syncthreads();
  double *T = scratch + b.offT;
  const int total = (int)min<int64_t>((int64_t)b.R * b.C, e0 + kGateChunk);
  for (int idx = (int)e0 + threadIdx.x; idx < total; idx += kThreads) {
    const int row = idx / b.C, col = idx - row * b.C;
    const int k1p = seg_of(b.rs, row), k2p = seg_of(b.cs, col);
    const int l = row - b.rs[k1p], r = col - b.cs[k2p];
    double acc = 0.0;
    for (int k1 = 0; k1 < 4; ++k1) {
      const int q = k1p * 4 + k1;
      const int64_t off = s_off[q];
      if (off < 0 || l >= s_rs[q][k1 + 1] - s_rs[q][k1]) continue;
      const double *Th = scratch + off + (int64_t)(s_rs[q][k1] + l) * s_C[q] + r;
      for (int k2 = 0; k2 < 4; ++k2) {
        const double g = sG[(k1p * 4 + k2p) * 16 + k1 * 4 + k2];
        if (g == 0.0 || r >= s_cs[q][k2 + 1] - s_cs[q][k2]) continue;
        acc += g * Th[s_cs[q][k2]];
      }
    }
    T[idx] = acc;
  }
}

// New A_a columns and A_{a+1} rows of one kept block (scatter); units: the
// chunks of the R x n columns, then those of the n x C rows, of which the
// first `kept` columns (rows) are written.
__global__ void __launch_bounds__(kThreads) k_split_gate(KetTables kt, int a, const Blk *blks, Units un,
                                                         const double *scratch, const double *scale) {
  const int bi = find_unit(un.first, un.n, blockIdx.x);
  const Blk &b = stage_block(blks, bi);
  const int pair = b.pair;
  double *A = kt.site[pair * kt.N + a];
  double *B = kt.site[pair * kt.N + a + 1];
  const int Dn = kt.dim(a + 1, pair), Dr = kt.dim(a + 2, pair);
  const double *U = scratch + b.offU, *Bo = scratch + b.offB;
  const int kept = b.kept;
  // units are counted for n kept vectors (the most a block can keep)
  const int u = blockIdx.x - un.first[bi], u1 = gate_chunks((int64_t)b.R * b.n);
  if (u < u1) {
    const int64_t e0 = (int64_t)u * kGateChunk, e1 = min<int64_t>((int64_t)b.R * kept, e0 + kGateChunk);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
      const int row = e / kept, jj = e - (int64_t)row * kept;
      const int k = seg_of(b.rs, row);
      const int l = kt.sec(a, pair, b.sa - qk_a(k), b.sb - qk_b(k)).x + (row - b.rs[k]);
      A[((int64_t)l * 4 + k) * Dn + b.j0 + jj] = U[(int64_t)jj * b.R + row];
    }
    return;
  }
  const int64_t e0 = (int64_t)(u - u1) * kGateChunk, e1 = min<int64_t>((int64_t)kept * b.C, e0 + kGateChunk);
  const double f = scale ? scale[pair] : 1.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
    const int jj = e / b.C, col = e - (int64_t)jj * b.C;
    const int k = seg_of(b.cs, col);
    const int r = kt.sec(a + 2, pair, b.sa + qk_a(k), b.sb + qk_b(k)).x + (col - b.cs[k]);
    B[((int64_t)(b.j0 + jj) * 4 + k) * Dr + r] = f * Bo[(int64_t)jj * b.C + col];
  }
}

// LQ move at site q: block = rows of sector s of bond q, columns (k, r).
// aux0 = offset of the sector in the (old) bond q.
__global__ void __launch_bounds__(kThreads) k_gather_lq(KetTables kt, int q, const Blk *blks, Units un,
                                                        double *scratch) {
  const int bi = find_unit(un.first, un.n, blockIdx.x);
  const Blk &b = stage_block(blks, bi);
  const int pair = b.pair;
  const double *A = kt.site[pair * kt.N + q];
  const int Dr = kt.dim(q + 1, pair);
  double *T = scratch + b.offT;
  const int64_t e0 = (int64_t)(blockIdx.x - un.first[bi]) * kGateChunk;
  const int64_t e1 = min<int64_t>((int64_t)b.R * b.C, e0 + kGateChunk);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
    const int row = e / b.C, col = e - (int64_t)row * b.C;
    const int k = seg_of(b.cs, col);
    const int r = kt.sec(q + 1, pair, b.sa + qk_a(k), b.sb + qk_b(k)).x + (col - b.cs[k]);
    T[e] = A[((int64_t)(b.aux0 + row) * 4 + k) * Dr + r];
  }
}

// A_q rows <- V^T rows; A_{q-1} columns <- old A_{q-1} U Sigma.
// aux0 = old offset of the sector in bond q, aux1 = old dimension of bond q.
// Units: chunks of the n x C new rows, then per local state k the tiles of
// the left neighbour's d_k x n product.
__global__ void __launch_bounds__(kThreads) k_apply_lq(KetTables kt, int q, const Blk *blks, Units un,
                                                       const double *scratch,
                                                       double *const *old_left) {
  const int bi = find_unit(un.first, un.n, blockIdx.x);
  const Blk &b = stage_block(blks, bi);
  const int pair = b.pair;
  double *A = kt.site[pair * kt.N + q];
  double *P = kt.site[pair * kt.N + q - 1];
  const double *Po = old_left[pair];
  const int Dr = kt.dim(q + 1, pair), Dn = kt.dim(q, pair);
  const int Dold = b.aux1, n = b.n;
  const double *U = scratch + b.offU, *Bo = scratch + b.offB, *S = scratch + b.offS;
  int u = blockIdx.x - un.first[bi];
  const int u1 = gate_chunks((int64_t)n * b.C);
  if (u < u1) {
    const int64_t e0 = (int64_t)u * kGateChunk, e1 = min<int64_t>((int64_t)n * b.C, e0 + kGateChunk);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
      const int jj = e / b.C, col = e - (int64_t)jj * b.C;
      const int k = seg_of(b.cs, col);
      const int r = kt.sec(q + 1, pair, b.sa + qk_a(k), b.sb + qk_b(k)).x + (col - b.cs[k]);
      const double s = S[jj];
      A[((int64_t)(b.j0 + jj) * 4 + k) * Dr + r] = s > 0.0 ? Bo[(int64_t)jj * b.C + col] / s : 0.0;
    }
    return;
  }
  u -= u1;
  // P[(l, k)][j0 + jj] = S[jj] sum_mm Po[(l, k)][aux0 + mm] U[jj][mm]
  __shared__ GemmTile sA, sB;
  for (int k = 0; k < 4; ++k) {
    const int2 ls = kt.sec(q - 1, pair, b.sa - qk_a(k), b.sb - qk_b(k));
    const int nt = gate_tiles(ls.y, n);
    if (u >= nt) {
      u -= nt;
      continue;
    }
    const double *Pk = Po + ((int64_t)ls.x * 4 + k) * Dold + b.aux0;
    double *Ck = P + ((int64_t)ls.x * 4 + k) * Dn + b.j0;
    const int R = b.R;
    gemm_tile_at<true>(
        sA, sB, ls.y, n, R, u, [&](int li, int mm) { return Pk[(int64_t)li * 4 * Dold + mm]; },
        [&](int mm, int jj) { return U[(int64_t)jj * R + mm]; },
        [&](int li, int jj, double v) { Ck[(int64_t)li * 4 * Dn + jj] = v * S[jj]; });
    return;
  }
}

// QR move at site p: block = rows (k, l) feeding sector s of bond p+1, columns r in s.
// aux0 = offset of the sector in the (old) bond p+1.
__global__ void __launch_bounds__(kThreads) k_gather_qr(KetTables kt, int p, const Blk *blks,
                                                        double *scratch) {
  const Blk &b = stage_block(blks, blockIdx.x);
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
  const Blk &b = stage_block(blks, blockIdx.x);
  const int pair = b.pair;
  double *A = kt.site[pair * kt.N + p];
  double *Nx = kt.site[pair * kt.N + p + 1];
  const double *No = old_right[pair];
  const int Dn = kt.dim(p + 1, pair), Drr = kt.dim(p + 2, pair);
  const int n = b.n;
  const double *U = scratch + b.offU, *Bo = scratch + b.offB;
  for (int64_t e = threadIdx.x; e < (int64_t)b.R * n; e += kThreads) {
    const int row = e / n, jj = e - (int64_t)row * n;
    const int k = seg_of(b.rs, row);
    const int l = kt.sec(p, pair, b.sa - qk_a(k), b.sb - qk_b(k)).x + (row - b.rs[k]);
    A[((int64_t)l * 4 + k) * Dn + b.j0 + jj] = U[(int64_t)jj * b.R + row];
  }
  // Nx[j0 + jj][x] = sum_mm B[jj][mm] No[aux0 + mm][x]
  const int W = 4 * Drr, Cb = b.C;
  const double *Nb = No + (int64_t)b.aux0 * W;
  double *Cn = Nx + (int64_t)b.j0 * W;
  block_gemm<false>(
      n, W, Cb, [&](int jj, int mm) { return Bo[(int64_t)jj * Cb + mm]; },
      [&](int mm, int x) { return Nb[(int64_t)mm * W + x]; },
      [&](int jj, int x, double v) { Cn[(int64_t)jj * W + x] = v; });
}

// Truncation of one ket per workgroup (App. A1: the largest singular values
// over all quantum-number blocks of the two-site matrix are kept).  With
// tot = sum s^2 over the ket's blocks, keep = min(chi, #{s^2 > tau tot}); a
// value is kept when its rank (larger values first, equal values in block
// order, then in order within the block) is below keep.  Each block's list
// is sorted, so its kept values are a prefix: the count and the block's
// offset j0 in the new bond go into the block, the kept counts per slot and
// their prefix sums into the bond's sector table, and (keep, discarded
// weight, relative gap at the cut) into stats[3 t ..].  The blocks of ket t
// are blks[kfirst[t] .. kfirst[t + 1]), in slot order.
constexpr int kSelThreads = 1024, kSelVals = 1;   // values per thread per pass
__device__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = kSelThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kSelThreads) k_select(Blk *blks, const int *kfirst, int maxv,
                                                     const double *scratch, int chi, double tau, KetTables kt,
                                                     int bond, int *kept_out, double *stats, double *scale) {
  extern __shared__ __align__(16) double sel_lds[];
  __shared__ double red[kSelThreads];
  __shared__ double s_th, s_so;
  const int t = blockIdx.x, i0 = kfirst[t], nb = kfirst[t + 1] - i0;
  double *v = sel_lds;                                    // [maxv] values in block order
  int *pre = reinterpret_cast<int *>(sel_lds + maxv);     // [nb + 1] value offsets of the blocks
  int *cnt = pre + nb + 1;                                // [nb] kept counts
  int *blk_of = cnt + nb;                                 // [nslot] block of a slot (-1: none)
  for (int i = threadIdx.x; i < nb; i += kSelThreads) {
    pre[i + 1] = blks[i0 + i].n;
    cnt[i] = 0;
  }
  for (int sl = threadIdx.x; sl < kt.nslot; sl += kSelThreads) blk_of[sl] = -1;
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += kSelThreads) blk_of[kt.slot(blks[i0 + i].sa, blks[i0 + i].sb)] = i;
  if (threadIdx.x == 0) {
    pre[0] = 0;
    for (int i = 0; i < nb; ++i) pre[i + 1] += pre[i];
    s_th = 0.0;
    s_so = 0.0;
  }
  __syncthreads();
  const int ntot = pre[nb];
  for (int e = threadIdx.x; e < ntot; e += kSelThreads) {
    int lo = 0, hi = nb;   // block of value e: pre[lo] <= e < pre[lo + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pre[mid] <= e) lo = mid;
      else hi = mid;
    }
    v[e] = scratch[blks[i0 + lo].offS + (e - pre[lo])];
  }
  __syncthreads();
  double part = 0.0;
  for (int e = threadIdx.x; e < ntot; e += kSelThreads) part += v[e] * v[e];
  const double tot = block_sum(part, red);
  double big = 0.0;
  for (int e = threadIdx.x; e < ntot; e += kSelThreads) big += (v[e] * v[e] > tau * tot) ? 1.0 : 0.0;
  const int keep = min(chi, (int)block_sum(big, red));
  // ranks: each thread takes kSelVals values per pass over all values
  double disc = 0.0;
  for (int e0 = 0; e0 < ntot; e0 += kSelVals * kSelThreads) {
    double x[kSelVals];
    int r[kSelVals];
#pragma unroll
    for (int u = 0; u < kSelVals; ++u) {
      const int e = e0 + u * kSelThreads + threadIdx.x;
      x[u] = e < ntot ? v[e] : 0.0;
      r[u] = 0;
    }
    const int eu = e0 + threadIdx.x;
    int f = 0;
    for (; f + 8 <= ntot; f += 8) {   // eight values per step: their LDS reads overlap
      double y[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) y[k] = v[f + k];
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int u = 0; u < kSelVals; ++u) r[u] += (y[k] > x[u] || (y[k] == x[u] && f + k < eu + u * kSelThreads)) ? 1 : 0;
    }
    for (; f < ntot; ++f) {
      const double y = v[f];
#pragma unroll
      for (int u = 0; u < kSelVals; ++u) r[u] += (y > x[u] || (y == x[u] && f < eu + u * kSelThreads)) ? 1 : 0;
    }
#pragma unroll
    for (int u = 0; u < kSelVals; ++u) {
      const int e = e0 + u * kSelThreads + threadIdx.x;
      if (e >= ntot) continue;
      if (r[u] < keep) {
        int lo = 0, hi = nb;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (pre[mid] <= e) lo = mid;
          else hi = mid;
        }
        atomicAdd(&cnt[lo], 1);
      } else {
        disc += x[u] * x[u];
      }
      if (r[u] == keep - 1) s_th = x[u];
      if (r[u] == keep) s_so = x[u];
    }
  }
  disc = block_sum(disc, red);
  // kept counts by slot and their prefix sums: the new bond's sector table
  if (threadIdx.x == 0) {
    int off = 0;
    for (int sl = 0; sl < kt.nslot; ++sl) {
      const int i = blk_of[sl];
      const int d = i >= 0 ? cnt[i] : 0;
      if (i >= 0) pre[i] = off;   // reused: offset j0 of block i
      kt.btab[((int64_t)bond * kt.npair + t) * kt.nslot + sl] = make_int2(off, d);
      off += d;
    }
    kt.bdim[bond * kt.npair + t] = off;
    stats[3 * t] = keep;
    stats[3 * t + 1] = disc;
    stats[3 * t + 2] = (keep > 0 && keep < ntot && s_th > 0.0) ? (s_th - s_so) / s_th : 1.0;
    // renormalisation: the kept values scaled back to the weight before the cut
    if (scale) scale[t] = (tot > disc && disc > 0.0) ? sqrt(tot / (tot - disc)) : 1.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += kSelThreads) {
    blks[i0 + i].kept = cnt[i];
    blks[i0 + i].j0 = pre[i];
    kept_out[i0 + i] = cnt[i];
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


// Exact centre moves by Householder QR, one workgroup per quantum-number
// block (App. A1, eq. orth_l / orth_r: a move only regauges the state).  The
// gathered block T (R x C, row-major) is factorised as X = Q_X R_X with
// X = T^T for a move to the left (LQ of T: L = R_X^T, rows of Q = Q_X^T) and
// X = T for a move to the right (QR of T).  X (m x c, k = min(m, c)) sits in
// LDS column by column; reflector j (H = I - tau v v^T, v_j = 1, LAPACK sign
// convention) is found by wave 0 and applied to the later columns by all
// waves, one column per wave at a time with a wave-wide reduction; Q_X is
// then formed in place from the reflectors (backward accumulation), with
// signs that make diag(R_X) non-negative.  Outputs,
// in the slots the move kernels read: U ([k][R]) and B ([k][C]) take R_X and
// Q_X^T (left move) or Q_X^T and R_X (right move); the k "singular values"
// are 1, so the apply kernels multiply by L (R_X) and write Q unscaled.
constexpr int kQrThreads = 1024, kQrWaves = kQrThreads / 64;

// one 64-bit value moved by a DPP lane permutation (two 32-bit moves)
template <int CTRL>
__device__ inline double qr_dpp64(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(x & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave, the same bits in every lane (each step
// adds two lanes' partial sums, and the two lanes of a step add the same
// operands): DPP within rows of 16 lanes, then two cross-row exchanges.
__device__ inline double wave_sum(double v) {
  v += qr_dpp64<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
  v += qr_dpp64<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
  v += qr_dpp64<0x141>(v);   // row_half_mirror: the other quad of 8
  v += qr_dpp64<0x140>(v);   // row_mirror: the other half of 16
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// (I - tj v v^T) applied to columns r0, r0 + kQrWaves, ... < rend of the
// m-row matrix X in LDS (v: x[j + 1 ..] with an implicit 1 at row j), two
// columns at a time so that their reductions overlap; one wave's part
__device__ inline void apply_reflector(double *qx, int m, int j, int r0, int rend, const double *x, double tj,
                                       int lane) {
  for (int r = r0; r < rend; r += 2 * kQrWaves) {
    const int r2 = r + kQrWaves;
    const bool two = r2 < rend;
    double *y = qx + (int64_t)r * m, *y2 = qx + (int64_t)(two ? r2 : r) * m;
    double w = lane == 0 ? y[j] : 0.0, w2 = (two && lane == 0) ? y2[j] : 0.0;
    for (int i = j + 1 + lane; i < m; i += 64) {
      const double xi = x[i];
      w += xi * y[i];
      if (two) w2 += xi * y2[i];
    }
    w = wave_sum(w) * tj;
    w2 = wave_sum(w2) * tj;
    if (lane == 0) {
      y[j] -= w;
      if (two) y2[j] -= w2;
    }
    for (int i = j + 1 + lane; i < m; i += 64) {
      const double xi = x[i];
      y[i] -= w * xi;
      if (two) y2[i] -= w2 * xi;
    }
  }
}

// column j of Q from the stored reflector j (v in x[j+1 ..], tau tj) once the
// later reflectors have been applied to it, by one wave
__device__ inline void form_q_column(double *qx, int m, int j, double tj, int lane) {
  double *x = qx + (int64_t)j * m;
  for (int i = j + 1 + lane; i < m; i += 64) x[i] *= -tj;
  for (int i = lane; i < j; i += 64) x[i] = 0.0;
  if (lane == 0) x[j] = 1.0 - tj;
}

// Householder reflector of column j of X (rows j..m-1) by one wave: tau[j],
// R_jj in x[j] and v (implicit 1 at row j) in x[j+1 ..]
__device__ inline void make_reflector(double *qx, int m, int j, int lane, double *tau) {
  double *x = qx + (int64_t)j * m;
  double sg = 0.0;
  for (int i = j + 1 + lane; i < m; i += 64) sg += x[i] * x[i];
  sg = wave_sum(sg);
  const double alpha = x[j];
  double t = 0.0, beta = alpha, scale = 0.0;
  if (sg > 0.0) {
    const double nrm = sqrt(alpha * alpha + sg);
    beta = alpha >= 0.0 ? -nrm : nrm;
    t = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  for (int i = j + 1 + lane; i < m; i += 64) x[i] *= scale;
  if (lane == 0) {
    tau[j] = t;
    x[j] = beta;
  }
}

__global__ void __launch_bounds__(kQrThreads) k_qr_blocks(const Blk *blks, const int *idx, double *scratch,
                                                          int left) {
  extern __shared__ __align__(16) double qx[];
  const Blk &b = stage_block(blks, idx[blockIdx.x]);
  const int R = b.R, C = b.C;
  const int m = left ? C : R, c = left ? R : C, k = min(m, c);
  double *tau = qx + (int64_t)m * c;
  const double *T = scratch + b.offT;
  for (int e = threadIdx.x; e < m * c; e += kQrThreads) {
    const int j = e / m, i = e - j * m;   // X(i, j)
    qx[e] = left ? T[(int64_t)j * C + i] : T[(int64_t)i * C + j];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // one barrier per reflector: wave 0, which owns column j + 1, updates it
  // first and forms reflector j + 1 while the other waves still apply j
  if (k > 0 && wave == 0) make_reflector(qx, m, 0, lane, tau);
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    const double *x = qx + (int64_t)j * m;
    const double tj = tau[j];
    if (wave == 0 && j + 1 < k) {
      if (tj != 0.0) apply_reflector(qx, m, j, j + 1, j + 2, x, tj, lane);
      make_reflector(qx, m, j + 1, lane, tau);
      if (tj != 0.0) apply_reflector(qx, m, j, j + 1 + kQrWaves, c, x, tj, lane);
    } else if (tj != 0.0) {
      apply_reflector(qx, m, j, j + 1 + wave, c, x, tj, lane);
    }
    __syncthreads();
  }
  double *Uo = scratch + b.offU, *Bo = scratch + b.offB, *So = scratch + b.offS;
  double *Rr = left ? Uo : Bo, *Qt = left ? Bo : Uo;
  // signs that make the diagonal of R_X non-negative (for a block of full
  // rank this fixes the factors, and with them the canonical form, uniquely)
  double *sgn = tau + k;
  for (int jj = threadIdx.x; jj < k; jj += kQrThreads) sgn[jj] = qx[(int64_t)jj * m + jj] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  for (int e = threadIdx.x; e < k * c; e += kQrThreads) {
    const int jj = e / c, r = e - jj * c;
    Rr[e] = r >= jj ? sgn[jj] * qx[(int64_t)r * m + jj] : 0.0;
  }
  for (int e = threadIdx.x; e < k; e += kQrThreads) So[e] = 1.0;
  __syncthreads();
  // Q_X (m x k) in place of the first k columns, backwards; column j + 1
  // becomes a column of Q (it is no longer read as reflector j + 1) in step j,
  // by wave 0, which then applies reflector j to it: one barrier per step
  for (int j = k - 1; j >= 0; --j) {
    const double *x = qx + (int64_t)j * m;
    if (wave == 0 && j + 1 < k) form_q_column(qx, m, j + 1, tau[j + 1], lane);
    apply_reflector(qx, m, j, j + 1 + wave, k, x, tau[j], lane);
    __syncthreads();
  }
  if (k > 0 && wave == 0) form_q_column(qx, m, 0, tau[0], lane);
  __syncthreads();
  for (int e = threadIdx.x; e < k * m; e += kQrThreads) Qt[e] = sgn[e / m] * qx[e];
}


// Entries of site x outside its quantum-number blocks set to zero, for every
// ket of the set (kernels that address a site by block never read them; a
// dense contraction does).  grid: (chunks, kets).
__global__ void k_mask_site(KetTables kt, int x) {
  const int pair = blockIdx.y;
  const int Dl = kt.dim(x, pair), Dr = kt.dim(x + 1, pair);
  double *A = kt.site[pair * kt.N + x];
  const int64_t tot = (int64_t)Dl * 4 * Dr;
  const int2 *tl = kt.btab + ((int64_t)x * kt.npair + pair) * kt.nslot;
  const int2 *tr = kt.btab + ((int64_t)(x + 1) * kt.npair + pair) * kt.nslot;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(e / (4 * Dr)), k = (int)((e / Dr) & 3), r = (int)(e % Dr);
    int sl = -1, sr = -1;
    for (int q = 0; q < kt.nslot; ++q) {
      if (l >= tl[q].x && l < tl[q].x + tl[q].y) sl = q;
      if (r >= tr[q].x && r < tr[q].x + tr[q].y) sr = q;
    }
    const int nb1 = kt.nb + 1;
    const bool ok = sl >= 0 && sr >= 0 && sr / nb1 == sl / nb1 + qk_a(k) && sr % nb1 == sl % nb1 + qk_b(k);
    if (!ok) A[e] = 0.0;
  }
}

}  // namespace

void launch_two_site(const KetTables &kt, int a, const Blk *blk, Units ug, const Blk *th, Units ut,
                     const int *thidx, const double *cs, double *gates, double *scratch, hipStream_t st) {
  hipLaunchKernelGGL(k_gates, dim3(kt.npair), dim3(256), 0, st, cs, gates);
  if (ut.total > 0) hipLaunchKernelGGL(k_theta, dim3(ut.total), dim3(kThreads), 0, st, kt, a, th, ut, scratch);
  if (ug.total > 0)
    hipLaunchKernelGGL(k_gate_gather, dim3(ug.total), dim3(kThreads), 0, st, kt, blk, ug, th, thidx, gates,
                       scratch);
}

void launch_split_gate(const KetTables &kt, int a, const Blk *blk, Units u, const double *scratch,
                       const double *scale, hipStream_t st) {
  if (u.total == 0) return;
  hipLaunchKernelGGL(k_split_gate, dim3(u.total), dim3(kThreads), 0, st, kt, a, blk, u, scratch, scale);
}

void launch_gather_lq(const KetTables &kt, int q, const Blk *blk, Units u, double *scratch,
                      hipStream_t st) {
  if (u.total == 0) return;
  hipLaunchKernelGGL(k_gather_lq, dim3(u.total), dim3(kThreads), 0, st, kt, q, blk, u, scratch);
}

void launch_apply_lq(const KetTables &kt, int q, const Blk *blk, Units u, const double *scratch,
                     double *const *old_left, hipStream_t st) {
  if (u.total == 0) return;
  hipLaunchKernelGGL(k_apply_lq, dim3(u.total), dim3(kThreads), 0, st, kt, q, blk, u, scratch, old_left);
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

void launch_select(Blk *blk, const int *kfirst, int nket, int maxv, const double *scratch, int chi, double tau,
                   const KetTables &kt, int bond, int *kept_out, double *stats, double *scale, hipStream_t st) {
  if (nket == 0) return;
  // once per process (thread-safe initialisation of a function-local static)
  static const bool attr_set = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_select),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kSelectLdsBytes);
    return true;
  }();
  (void)attr_set;
  const size_t lds = select_lds_bytes(maxv, kt.nslot);
  hipLaunchKernelGGL(k_select, dim3(nket), dim3(kSelThreads), lds, st, blk, kfirst, maxv, scratch, chi, tau, kt,
                     bond, kept_out, stats, scale);
}

void launch_qr_blocks(const Blk *blk, const int *idx, int nblk, int lds_bytes, bool left, double *scratch,
                      hipStream_t st) {
  if (nblk == 0) return;
  static const bool attr_set = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_qr_blocks),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kQrLdsBytes);
    return true;
  }();
  (void)attr_set;
  hipLaunchKernelGGL(k_qr_blocks, dim3(nblk), dim3(kQrThreads), lds_bytes, st, blk, idx, scratch, left ? 1 : 0);
}

void launch_mask_site(const KetTables &kt, int x, int max_elems, hipStream_t st) {
  if (kt.npair == 0 || max_elems <= 0) return;
  const int chunks = std::min(1024, (max_elems + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_mask_site, dim3(chunks, kt.npair), dim3(kThreads), 0, st, kt, x);
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
